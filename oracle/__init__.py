"""Plain FP64 CPU oracle (ctypes wrapper around ``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU baseline
leg of the benchmark load this package; the GPU engine never does, and this
package imports nothing from the engine.  All arrays are float64 numpy arrays
in original particle order (``x`` is (N, 3), ``q`` is (N, 4) Hamilton
quaternions (w, x, y, z)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.c")]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (-O2, no FMA contraction, OpenMP
    per-particle loops)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-D_DEFAULT_SOURCE", "-o", LIB_PATH + ".tmp"] + SOURCES + ["-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


class PatchyParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("sigma", ctypes.c_double),
                ("rcut", ctypes.c_double), ("eps_p", ctypes.c_double),
                ("w", ctypes.c_double), ("delta", ctypes.c_double),
                ("rpc", ctypes.c_double), ("model", ctypes.c_int)]


class RunParams(ctypes.Structure):
    _fields_ = [("pot", ctypes.c_int), ("mass", ctypes.c_double),
                ("inertia", ctypes.c_double), ("dt", ctypes.c_double),
                ("skin", ctypes.c_double), ("eps", ctypes.c_double),
                ("sigma", ctypes.c_double), ("rcut", ctypes.c_double),
                ("patchy", PatchyParams)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.or_min_image.restype = ctypes.c_double
        L.or_min_image.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_max_threads.restype = ctypes.c_int
        L.or_max_threads.argtypes = []
        L.or_patchy_pair_scales.restype = None
        L.or_patchy_pair_scales.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double,
                                            ctypes.POINTER(PatchyParams), ctypes.c_int, _D, _D]
        for name in ("or_pairs_brute", "or_pairs_cells"):
            f = getattr(L, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_double, _I, ctypes.c_int64]
        L.or_neighbors_of.restype = ctypes.c_int
        L.or_neighbors_of.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_double,
                                      ctypes.c_double, _I, ctypes.c_int]
        L.or_pair_margin.restype = ctypes.c_double
        L.or_pair_margin.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, ctypes.c_int]
        L.or_lj_pair.restype = ctypes.c_double
        L.or_lj_pair.argtypes = [ctypes.c_double] * 4 + [_D]
        L.or_lj_forces.restype = None
        L.or_lj_forces.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, _D, _D, _D, _D,
                                   _D]
        L.or_lj_force_one.restype = None
        L.or_lj_force_one.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
        L.or_quat_to_matrix.restype = None
        L.or_quat_to_matrix.argtypes = [_D, _D]
        L.or_patchy_pair.restype = ctypes.c_double
        L.or_patchy_pair.argtypes = [_D, _D, _D, _D, ctypes.c_double,
                                     ctypes.POINTER(PatchyParams), _D, _D, _D]
        L.or_patchy_forces.restype = None
        L.or_patchy_forces.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double,
                                       ctypes.POINTER(PatchyParams), ctypes.c_int, _D, _D, _D, _D,
                                       _D, _D]
        _U64P = ctypes.POINTER(ctypes.c_uint64)
        L.or_philox4x64.argtypes = [_U64P, _U64P, _U64P]
        L.or_thermostat.restype = ctypes.c_int
        L.or_thermostat.argtypes = [ctypes.c_int, _D, _D] + [ctypes.c_double] * 4 + \
            [ctypes.c_uint64, ctypes.c_uint64]
        L.or_run.restype = ctypes.c_int
        L.or_run.argtypes = [ctypes.c_int, _D, _D, _D, _D, ctypes.c_double,
                             ctypes.POINTER(RunParams), ctypes.c_int, _D, _I, ctypes.c_int, _D]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


@dataclass
class LJ:
    """Truncated-and-shifted Lennard-Jones parameters (Eq. 1)."""
    eps: float = 1.0
    sigma: float = 1.0
    rcut: float = 2.5


@dataclass
class Patchy:
    """Patchy model parameters (readings stated in oracle.c): model 0 is the
    four-patch variant (defaults), model 1 the paper's two-patch model (use
    Patchy.paper())."""
    eps: float = 1.0
    sigma: float = 1.0
    rcut: float = 1.5
    eps_p: float = 1.0
    w: float = 0.12
    delta: float = 0.5
    rpc: float = 0.75
    model: int = 0

    @staticmethod
    def paper() -> "Patchy":
        """Two polar patches, (sigma/r)^200 core, patch range 0.18 sigma."""
        return Patchy(eps=1.0, sigma=1.0, rcut=1.18, eps_p=1.0, w=0.12, delta=0.5, rpc=0.18,
                      model=1)

    def c(self) -> PatchyParams:
        return PatchyParams(self.eps, self.sigma, self.rcut, self.eps_p, self.w,
                            self.delta, self.rpc, self.model)


def min_image(d: float, L: float) -> float:
    return lib().or_min_image(d, L)


def pairs(x, L, rv, method="cells"):
    """Sorted (P, 2) int32 array of unordered pairs i<j with r < rv."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    f = lib().or_pairs_cells if method == "cells" else lib().or_pairs_brute
    cnt = f(n, _d(x), L, rv, None, 0)
    out = np.zeros((max(cnt, 1), 2), dtype=np.int32)
    f(n, _d(x), L, rv, out.ctypes.data_as(_I), cnt)
    out = out[:cnt]
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def neighbors_of(i, x, L, rv):
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    cnt = lib().or_neighbors_of(i, n, _d(x), L, rv, None, 0)
    out = np.zeros(max(cnt, 1), dtype=np.int32)
    lib().or_neighbors_of(i, n, _d(x), L, rv, out.ctypes.data_as(_I), cnt)
    return out[:cnt]


def pair_margin(x, L, radii):
    x = _f64(x, (-1, 3))
    r = _f64(radii)
    return lib().or_pair_margin(x.shape[0], _d(x), L, _d(r), len(r))


def lj_pair(r2, p: LJ):
    fs = ctypes.c_double()
    v = lib().or_lj_pair(r2, p.eps, p.sigma, p.rcut, ctypes.byref(fs))
    return v, fs.value


def lj_forces(x, L, p: LJ, use_cells=True, with_abs=False, with_eabs=False):
    """(F (N,3), e (N,), w (N,)[, Fabs (N,3)][, Eabs (N,)]) summed over all j
    with r < rcut; Fabs and Eabs are the term-magnitude scales of F and e."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    F = np.zeros((n, 3))
    e = np.zeros(n)
    w = np.zeros(n)
    A = np.zeros((n, 3))
    EA = np.zeros(n)
    lib().or_lj_forces(n, _d(x), L, p.eps, p.sigma, p.rcut, int(use_cells), _d(F), _d(e),
                       _d(w), _d(A), _d(EA))
    out = (F, e, w)
    if with_abs:
        out += (A,)
    if with_eabs:
        out += (EA,)
    return out


def lj_force_one(i, x, L, p: LJ):
    x = _f64(x, (-1, 3))
    f = np.zeros(3)
    e = ctypes.c_double()
    lib().or_lj_force_one(i, x.shape[0], _d(x), L, p.eps, p.sigma, p.rcut, _d(f), ctypes.byref(e))
    return f, e.value


def quat_to_matrix(q):
    q = _f64(q)
    R = np.zeros(9)
    lib().or_quat_to_matrix(_d(q), _d(R))
    return R.reshape(3, 3)


def patchy_pair(xi, xj, qi, qj, L, p: Patchy):
    """(V, F_j, tau_i, tau_j) for one pair."""
    xi, xj, qi, qj = _f64(xi), _f64(xj), _f64(qi), _f64(qj)
    Fj, ti, tj = np.zeros(3), np.zeros(3), np.zeros(3)
    pc = p.c()
    v = lib().or_patchy_pair(_d(xi), _d(xj), _d(qi), _d(qj), L, ctypes.byref(pc),
                             _d(Fj), _d(ti), _d(tj))
    return v, Fj, ti, tj


def patchy_forces(x, q, L, p: Patchy, use_cells=True, with_abs=False):
    """(F, T, e, w[, Fabs, Tabs]) summed over all pairs."""
    x = _f64(x, (-1, 3))
    q = _f64(q, (-1, 4))
    n = x.shape[0]
    F, T = np.zeros((n, 3)), np.zeros((n, 3))
    e, w = np.zeros(n), np.zeros(n)
    FA, TA = np.zeros((n, 3)), np.zeros((n, 3))
    pc = p.c()
    lib().or_patchy_forces(n, _d(x), _d(q), L, ctypes.byref(pc), int(use_cells),
                           _d(F), _d(T), _d(e), _d(w), _d(FA), _d(TA))
    return (F, T, e, w, FA, TA) if with_abs else (F, T, e, w)


def patchy_pair_scales(x, q, L, p: Patchy, use_cells=True):
    """(Fpair (N,3), Tpair (N,3)): per component sum_j |F_i(ij)| and
    sum_j |tau_i(ij)| over the pairs of i -- the magnitudes of the net pair
    force and torque, where patchy_forces' Fabs / Tabs sum the magnitudes of
    the individual terms of each pair."""
    x = _f64(x, (-1, 3))
    q = _f64(q, (-1, 4))
    n = x.shape[0]
    FP, TP = np.zeros((n, 3)), np.zeros((n, 3))
    pc = p.c()
    lib().or_patchy_pair_scales(n, _d(x), _d(q), L, ctypes.byref(pc), int(use_cells),
                                _d(FP), _d(TP))
    return FP, TP


def set_threads(threads: int) -> None:
    """Threads of the oracle's OpenMP per-particle force loops (results are
    bitwise independent of the count)."""
    lib().or_set_threads(int(threads))


def max_threads() -> int:
    return int(lib().or_max_threads())


def run(x, v, L, *, pot, nsteps, dt, skin, mass=1.0, inertia=1.0, lj: LJ | None = None,
        patchy: Patchy | None = None, q=None, angmom=None, rb_cap=100000):
    """Velocity Verlet run.  Returns dict with final x, v (q, angmom), energies
    (nsteps+1, 3) = (E_kin, E_pot, virial), rebuild steps and displacement margin."""
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    n = x.shape[0]
    rp = RunParams()
    rp.pot = 0 if pot == "lj" else 1
    rp.mass, rp.inertia, rp.dt, rp.skin = mass, inertia, dt, skin
    if rp.pot == 0:
        lj = lj or LJ()
        rp.eps, rp.sigma, rp.rcut = lj.eps, lj.sigma, lj.rcut
        qq = np.zeros((n, 4))
        qq[:, 0] = 1
        am = np.zeros((n, 3))
    else:
        patchy = patchy or Patchy()
        rp.eps, rp.sigma, rp.rcut = patchy.eps, patchy.sigma, patchy.rcut
        rp.patchy = patchy.c()
        qq = _f64(q, (-1, 4)).copy()
        am = _f64(angmom, (-1, 3)).copy()
    en = np.zeros((nsteps + 1, 3))
    rb = np.zeros(rb_cap, dtype=np.int32)
    margin = ctypes.c_double()
    nrb = lib().or_run(n, _d(x), _d(v), _d(qq), _d(am), L, ctypes.byref(rp), nsteps,
                       _d(en), rb.ctypes.data_as(_I), rb_cap, ctypes.byref(margin))
    out = dict(x=x, v=v, energies=en, rebuild_steps=rb[:min(nrb, rb_cap)].copy(),
               disp_margin=margin.value)
    if rp.pot == 1:
        out["q"] = qq
        out["angmom"] = am
    return out


def philox4x64(ctr, key):
    """Philox4x64-10 block: four uint64 words from a 4-word counter and a
    2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    kk = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    P = ctypes.POINTER(ctypes.c_uint64)
    lib().or_philox4x64(c.ctypes.data_as(P), kk.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def thermostat(v, angmom, T, prob, seed, counter, mass=1.0, inertia=1.0):
    """(v', angmom', refreshed) after one thermostat application (or_thermostat);
    the inputs are not modified.  angmom may be None."""
    v2 = np.array(v, dtype=np.float64, order="C", copy=True)
    a2 = None if angmom is None else np.array(angmom, dtype=np.float64, order="C", copy=True)
    n = v2.shape[0]
    hits = lib().or_thermostat(n, _d(v2), _d(a2) if a2 is not None else None, T, mass, inertia,
                               prob, seed, counter)
    return v2, a2, hits
