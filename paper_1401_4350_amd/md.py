"""Thin ctypes binding of libmd.so (include/md.h).

Argument marshalling only: every step of the force path runs in the HIP
kernels behind the C ABI.  PyTorch provides the two device buffers and the
stream.  Importing this module loads libmd.so and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1401_4350_amd.build` "
        "(the engine has no fallback path)")

# torch first: libmd.so then binds to the HIP runtime torch has already loaded
_lib = ctypes.CDLL(LIB_PATH)

MD_OK = 0
MODE = {"vertex": 0, "edge": 1, "newton": 2, "edge_det": 3}
POT = {"lj": 0, "patchy": 1}
PREC = {"fp64": 0, "fp32": 1, "fp32_kahan": 2}


class MDParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pot", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("max_neighbors", ctypes.c_int32), ("box", ctypes.c_double),
                ("eps", ctypes.c_double), ("sigma", ctypes.c_double),
                ("rcut", ctypes.c_double), ("skin", ctypes.c_double),
                ("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("eps_p", ctypes.c_double), ("patch_w", ctypes.c_double),
                ("patch_delta", ctypes.c_double), ("patch_rcut", ctypes.c_double),
                ("inertia", ctypes.c_double), ("newton_m", ctypes.c_int32),
                ("edge_store", ctypes.c_int32), ("cell_order", ctypes.c_int32),
                ("patch_model", ctypes.c_int32)]


class MDSizes(ctypes.Structure):
    _fields_ = [("state_bytes", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("alignment", ctypes.c_uint64)]


class MDStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("rebuilds", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("max_list_len", ctypes.c_int32),
                ("n_cells", ctypes.c_int32), ("tiles_total", ctypes.c_int32),
                ("tiles_staged", ctypes.c_int32), ("nonzero_pairs", ctypes.c_int64)]


class MDProfile(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("integrate_ms", ctypes.c_double),
                ("rebuild_ms", ctypes.c_double), ("force_ms", ctypes.c_double),
                ("kick_ms", ctypes.c_double)]


class MDBatchParams(ctypes.Structure):
    _fields_ = [("max_systems", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("max_particles", ctypes.c_int64), ("pool_bytes", ctypes.c_uint64)]


class MDBatchInfo(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("lds_cap", ctypes.c_int32),
                ("particles", ctypes.c_int64), ("bytes", ctypes.c_uint64),
                ("launches", ctypes.c_int64), ("captures", ctypes.c_int64),
                ("regrids", ctypes.c_int64)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_sys_p = ctypes.c_void_p
_bat_p = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "md_query_sizes": ([ctypes.POINTER(MDParams), ctypes.POINTER(MDSizes)], ctypes.c_int),
    "md_cell_order_ranks": ([ctypes.c_int32, ctypes.c_int32, _I32P], ctypes.c_int),
    "md_create": ([ctypes.POINTER(MDParams), _P, ctypes.c_uint64, _P, ctypes.c_uint64, _P,
                   ctypes.POINTER(_sys_p)], ctypes.c_int),
    "md_set_state": ([_sys_p, _D, _D, _D, _D], ctypes.c_int),
    "md_build_cells": ([_sys_p], ctypes.c_int),
    "md_build_neighbors": ([_sys_p], ctypes.c_int),
    "md_forces": ([_sys_p, ctypes.c_int32], ctypes.c_int),
    "md_step": ([_sys_p, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "md_energy": ([_sys_p, _D, _D, _D], ctypes.c_int),
    "md_particle_energies": ([_sys_p, _D], ctypes.c_int),
    "md_thermostat": ([_sys_p, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                       ctypes.c_uint64], ctypes.c_int),
    "md_get_state": ([_sys_p, _D, _D, _D, _D, _D, _D], ctypes.c_int),
    "md_get_pairs": ([_sys_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                      ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "md_stats": ([_sys_p, ctypes.POINTER(MDStats)], ctypes.c_int),
    "md_profile_enable": ([_sys_p, ctypes.c_int32], ctypes.c_int),
    "md_profile_read": ([_sys_p, ctypes.POINTER(MDProfile)], ctypes.c_int),
    "md_destroy": ([_sys_p], None),
    "md_status_str": ([ctypes.c_int32], ctypes.c_char_p),
    "md_last_error": ([_sys_p], ctypes.c_char_p),
    "md_batch_query_sizes": ([ctypes.POINTER(MDBatchParams), ctypes.POINTER(ctypes.c_uint64)],
                             ctypes.c_int),
    "md_batch_create": ([ctypes.POINTER(MDBatchParams), _P, ctypes.c_uint64, _P,
                         ctypes.POINTER(_bat_p)], ctypes.c_int),
    "md_batch_admit": ([_bat_p, _sys_p, ctypes.c_int64, _I32P], ctypes.c_int),
    "md_batch_step": ([_bat_p, _I32P], ctypes.c_int),
    "md_batch_steps_left": ([_bat_p, ctypes.c_int32, _I64P], ctypes.c_int),
    "md_batch_retire": ([_bat_p, ctypes.c_int32], ctypes.c_int),
    "md_batch_sync": ([_bat_p], ctypes.c_int),
    "md_batch_thermostat": ([_bat_p, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                             ctypes.c_uint64, ctypes.c_uint64], ctypes.c_int),
    "md_batch_info": ([_bat_p, ctypes.POINTER(MDBatchInfo)], ctypes.c_int),
    "md_batch_destroy": ([_bat_p], None),
    "md_batch_last_error": ([_bat_p], ctypes.c_char_p),
    "md_forces_static": ([ctypes.POINTER(MDParams), _P, _P, _P, _P, ctypes.c_int32, _P, _P],
                         ctypes.c_int),
}
# MD_STATIC_SCRATCH_BYTES of include/md.h
STATIC_SCRATCH_BYTES = 64 << 20
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class MDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.md_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


CELL_ORDER = {"row_major": 0, "row_major_gather": 1, "morton": 2, "hilbert": 3}
PATCH_MODEL = {"tetra": 0, "polar2": 1}


def make_params(w, prec: str = "fp64", newton_m: int = 0, edge_store: bool = False,
                cell_order: str = "row_major") -> MDParams:
    """md_params from a Workload of paper_1401_4350_amd.inputs; newton_m is
    the number of replicated force arrays of the Newton mode (0: LDS);
    edge_store reserves the per-edge arrays of the deterministic edge mode;
    cell_order is the slot order of the cells (CELL_ORDER)."""
    p = MDParams()
    p.newton_m = newton_m
    p.edge_store = int(edge_store)
    p.cell_order = CELL_ORDER[cell_order]
    p.n, p.pot, p.prec = w.n, POT[w.pot], PREC[prec]
    p.max_neighbors = w.list_capacity()
    p.box, p.eps, p.sigma, p.rcut, p.skin = w.box, w.eps, w.sigma, w.rcut, w.skin
    p.mass, p.dt = w.mass, w.dt
    p.eps_p, p.patch_w, p.patch_delta = w.eps_p, w.patch_w, w.patch_delta
    p.patch_rcut, p.inertia = w.patch_rcut, w.inertia
    p.patch_model = PATCH_MODEL[w.patch_model] if w.pot == "patchy" else 0
    return p


def cell_order_ranks(nc: int, order: str) -> np.ndarray:
    """Position of every cell of an nc^3 grid (row-major index) in the given
    cell order (md_cell_order_ranks)."""
    out = np.zeros(nc ** 3, dtype=np.int32)
    st = _lib.md_cell_order_ranks(nc, CELL_ORDER[order], out.ctypes.data_as(_I32P))
    if st != MD_OK:
        raise MDError(st, "md_cell_order_ranks")
    return out


def query_sizes(p: MDParams) -> MDSizes:
    s = MDSizes()
    st = _lib.md_query_sizes(ctypes.byref(p), ctypes.byref(s))
    if st != MD_OK:
        raise MDError(st, "md_query_sizes")
    return s


def forces_static(params: MDParams, x: torch.Tensor, q: torch.Tensor | None = None,
                  mode: str = "vertex", stream: torch.cuda.Stream | None = None):
    """md_forces_static: forces (and torques) of the device coordinates x
    (n x 3 float64 on the current device; q n x 4 for patchy) with no
    workspace.  The outputs and the status word are allocated here, by the
    caller's side; the call itself allocates nothing.  Returns
    (f, torque or None, status tensor); the status holds MD_OK or a device
    error code once the stream has run the call."""
    n = params.n
    dev = torch.device("cuda", torch.cuda.current_device())
    patchy = params.pot == POT["patchy"]
    for name, a, cols in (("x", x, 3), ("q", q, 4)):
        if a is None:
            continue
        if a.dtype != torch.float64 or a.device != dev or tuple(a.shape) != (n, cols) \
                or not a.is_contiguous():
            raise ValueError(f"{name} must be a contiguous ({n}, {cols}) float64 tensor on {dev}")
    f = torch.empty((n, 3), dtype=torch.float64, device=dev)
    t = torch.empty((n, 3), dtype=torch.float64, device=dev) if patchy else None
    status = torch.full((1,), -100, dtype=torch.int32, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = _lib.md_forces_static(ctypes.byref(params), ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(q.data_ptr() if q is not None else 0),
                               ctypes.c_void_p(f.data_ptr()),
                               ctypes.c_void_p(t.data_ptr() if t is not None else 0),
                               MODE[mode], ctypes.c_void_p(status.data_ptr()),
                               ctypes.c_void_p(s.cuda_stream))
    if st != MD_OK:
        raise MDError(st, "md_forces_static")
    return f, t, status


class System:
    """One simulated system on the current HIP device (see include/md.h)."""

    def __init__(self, params: MDParams, stream: torch.cuda.Stream | None = None):
        self.params = params
        self.n = params.n
        self.patchy = params.pot == POT["patchy"]
        sz = query_sizes(params)
        dev = torch.device("cuda", torch.cuda.current_device())
        a = int(sz.alignment)
        # over-allocate by one alignment unit and align the base pointer
        self._state = torch.empty(int(sz.state_bytes) + a, dtype=torch.uint8, device=dev)
        sp = (self._state.data_ptr() + a - 1) // a * a
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _sys_p()
        self._ws = torch.empty(int(sz.workspace_bytes) + a, dtype=torch.uint8, device=dev)
        wp = (self._ws.data_ptr() + a - 1) // a * a
        st = _lib.md_create(ctypes.byref(params), sp, sz.state_bytes, wp, sz.workspace_bytes,
                            self.stream.cuda_stream, ctypes.byref(h))
        if st != MD_OK:
            raise MDError(st, "md_create")
        self._h = h
        self.state_bytes = int(sz.state_bytes)
        self.workspace_bytes = int(sz.workspace_bytes)

    def _check(self, st, what):
        if st != MD_OK:
            raise MDError(st, f"{what}: {_lib.md_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            _lib.md_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ---------------------------------------------------------------
    def set_state(self, x, v, q=None, angmom=None):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.n, 3)
        if self.patchy:
            q = np.ascontiguousarray(q, dtype=np.float64).reshape(self.n, 4)
            angmom = np.ascontiguousarray(angmom, dtype=np.float64).reshape(self.n, 3)
        else:
            q = angmom = None
        self._check(_lib.md_set_state(self._h, _dp(x), _dp(v), _dp(q), _dp(angmom)),
                    "md_set_state")

    def build_cells(self):
        self._check(_lib.md_build_cells(self._h), "md_build_cells")

    def build_neighbors(self):
        self._check(_lib.md_build_neighbors(self._h), "md_build_neighbors")

    def build(self):
        self.build_cells()
        self.build_neighbors()

    def forces(self, mode: str = "vertex"):
        self._check(_lib.md_forces(self._h, MODE[mode]), "md_forces")

    def step(self, nsteps: int, mode: str = "vertex"):
        self._check(_lib.md_step(self._h, nsteps, MODE[mode]), "md_step")

    def thermostat(self, temperature: float, prob: float, seed: int, counter: int):
        """md_thermostat: redraw momenta with probability prob at temperature."""
        self._check(_lib.md_thermostat(self._h, temperature, prob, seed, counter),
                    "md_thermostat")

    def energy(self):
        k, p, w = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(_lib.md_energy(self._h, ctypes.byref(k), ctypes.byref(p), ctypes.byref(w)),
                    "md_energy")
        return k.value, p.value, w.value

    def particle_energies(self):
        e = np.zeros(self.n)
        self._check(_lib.md_particle_energies(self._h, _dp(e)), "md_particle_energies")
        return e

    def get_state(self):
        n = self.n
        out = {k: np.zeros((n, 3)) for k in ("x", "v", "f")}
        if self.patchy:
            out["q"] = np.zeros((n, 4))
            out["angmom"] = np.zeros((n, 3))
            out["torque"] = np.zeros((n, 3))
        self._check(_lib.md_get_state(self._h, _dp(out["x"]), _dp(out["v"]), _dp(out["f"]),
                                      _dp(out.get("q")), _dp(out.get("angmom")),
                                      _dp(out.get("torque"))), "md_get_state")
        return out

    def pairs(self):
        """Half list in original ids, sorted, as an (|E|, 2) int32 array."""
        cnt = ctypes.c_int64()
        self._check(_lib.md_get_pairs(self._h, None, 0, ctypes.byref(cnt)), "md_get_pairs")
        out = np.zeros((max(cnt.value, 1), 2), dtype=np.int32)
        self._check(_lib.md_get_pairs(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      cnt.value, ctypes.byref(cnt)), "md_get_pairs")
        out = out[:cnt.value]
        return out[np.lexsort((out[:, 1], out[:, 0]))]

    def profile(self, on: bool = True):
        self._check(_lib.md_profile_enable(self._h, int(on)), "md_profile_enable")

    def profile_read(self) -> dict:
        p = MDProfile()
        self._check(_lib.md_profile_read(self._h, ctypes.byref(p)), "md_profile_read")
        return dict(steps=p.steps, integrate_ms=p.integrate_ms, rebuild_ms=p.rebuild_ms,
                    force_ms=p.force_ms, kick_ms=p.kick_ms)

    def stats(self) -> dict:
        s = MDStats()
        self._check(_lib.md_stats(self._h, ctypes.byref(s)), "md_stats")
        return dict(steps=s.steps, rebuilds=s.rebuilds, pairs=s.pairs,
                    max_list_len=s.max_list_len, n_cells=s.n_cells,
                    tiles_total=s.tiles_total, tiles_staged=s.tiles_staged,
                    nonzero_pairs=s.nonzero_pairs)


def batch_params(max_systems: int, max_particles: int, pool_bytes: int, mode: str = "vertex",
                 steps_per_launch: int = 64, use_graph: bool = True) -> MDBatchParams:
    p = MDBatchParams()
    p.max_systems, p.mode, p.steps_per_launch = max_systems, MODE[mode], steps_per_launch
    p.use_graph, p.max_particles, p.pool_bytes = int(use_graph), max_particles, pool_bytes
    return p


def batch_workspace_bytes(p: MDBatchParams) -> int:
    b = ctypes.c_uint64()
    st = _lib.md_batch_query_sizes(ctypes.byref(p), ctypes.byref(b))
    if st != MD_OK:
        raise MDError(st, "md_batch_query_sizes")
    return int(b.value)


class Batch:
    """Batched serving handle (md_batch_* in include/md.h).  Holds a reference
    to every admitted System so its buffers outlive the admission."""

    def __init__(self, params: MDBatchParams, stream: torch.cuda.Stream | None = None):
        self.params = params
        nbytes = batch_workspace_bytes(params)
        dev = torch.device("cuda", torch.cuda.current_device())
        a = 256
        self._ws = torch.empty(nbytes + a, dtype=torch.uint8, device=dev)
        wp = (self._ws.data_ptr() + a - 1) // a * a
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _bat_p()
        st = _lib.md_batch_create(ctypes.byref(params), wp, nbytes, self.stream.cuda_stream,
                                  ctypes.byref(h))
        if st != MD_OK:
            raise MDError(st, "md_batch_create")
        self._h = h
        self.systems: dict[int, System] = {}

    def _check(self, st, what):
        if st != MD_OK:
            raise MDError(st, f"{what}: {_lib.md_batch_last_error(self._h).decode()}")

    def admit(self, system: System, nsteps: int) -> int:
        slot = ctypes.c_int32()
        self._check(_lib.md_batch_admit(self._h, system._h, nsteps, ctypes.byref(slot)),
                    "md_batch_admit")
        self.systems[slot.value] = system
        return slot.value

    def try_admit(self, system: System, nsteps: int) -> int | None:
        """Slot, or None when the batch has no room (MD_ERR_BUFFER_TOO_SMALL)."""
        try:
            return self.admit(system, nsteps)
        except MDError as e:
            if e.status == -2:
                return None
            raise

    def step(self) -> int:
        k = ctypes.c_int32()
        self._check(_lib.md_batch_step(self._h, ctypes.byref(k)), "md_batch_step")
        return k.value

    def steps_left(self, slot: int) -> int:
        v = ctypes.c_int64()
        self._check(_lib.md_batch_steps_left(self._h, slot, ctypes.byref(v)), "md_batch_steps_left")
        return v.value

    def retire(self, slot: int) -> System:
        """Frees the slot and returns its System; raises MDError with the
        system's device status (the slot is freed all the same) or for a free
        slot."""
        st = _lib.md_batch_retire(self._h, slot)
        system = self.systems.pop(slot, None) if self.steps_left(slot) == -1 else None
        self._check(st, "md_batch_retire")
        return system

    def sync(self):
        self._check(_lib.md_batch_sync(self._h), "md_batch_sync")

    def thermostat(self, slot: int, temperature: float, prob: float, seed: int, counter: int):
        """md_batch_thermostat: the momentum refresh of an admitted system,
        before the next batch step."""
        self._check(_lib.md_batch_thermostat(self._h, slot, temperature, prob, seed, counter),
                    "md_batch_thermostat")

    def info(self) -> dict:
        i = MDBatchInfo()
        self._check(_lib.md_batch_info(self._h, ctypes.byref(i)), "md_batch_info")
        return dict(active=i.active, lds_cap=i.lds_cap, particles=i.particles, bytes=i.bytes,
                    launches=i.launches, captures=i.captures, regrids=i.regrids)

    def close(self):
        if getattr(self, "_h", None):
            _lib.md_batch_destroy(self._h)
            self._h = None
            self.systems.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lib():
    return _lib
