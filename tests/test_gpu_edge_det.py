"""GPU parity, deterministic edge mode: one thread per half-list entry stores
the pair's result per edge, one thread per particle sums its edges' results in
the order of its list (through the C ABI), against the FP64 oracle, and its
bitwise reproducibility.

Bars as for the atomic edge mode (FP64 forces and torques within 1e-10 of the
sum of term magnitudes per component, FP32 pair maths within 1e-5, 100 steps
within 1e-9), plus: repeated force calls, and two systems stepped from the
same state, agree bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS

from _helpers import accepted_state, cond_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import md as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def det_system(md, w, s, prec="fp64"):
    g = md.System(md.make_params(w, prec, edge_store=True))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    return g


def patchy_params(w):
    return oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                         delta=w.patch_delta, rpc=w.patch_rcut)


LJ_CASES = {
    "lj4096": ("lj_small", {}),                       # staged tiles
    "lj1000_ragged": ("lj_small", {"n": 1000}),
    "lj300_two_cells": ("lj_small", {"n": 300}),      # 2 cells per side: global gathers
    "lj_dilute": ("lj_small", {"n": 2000, "rho": 0.1}),
    "lj_dense_rc3": ("lj_many_dense", {"n": 3000}),
}


@pytest.mark.parametrize("case", list(LJ_CASES))
def test_lj_forces_fp64(md, case):
    name, over = LJ_CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 2)
    say(f"[edge_det lj fp64] {case} n={w.n}")
    g = det_system(md, w, s)
    g.forces("edge_det")
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
    assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "fp32_kahan"])
def test_lj_forces_fp32(md, prec):
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 4)
    say(f"[edge_det lj {prec}]")
    g = det_system(md, w, s, prec=prec)
    g.forces("edge_det")
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_abs=True)
    assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-5


@pytest.mark.parametrize("over", [{"n": 3000}, {"n": 200, "rho": 0.5}])
def test_patchy_forces_torques_fp64(md, over):
    w = WORKLOADS["patchy"].with_(**over)
    s = accepted_state(w, 2)
    say(f"[edge_det patchy fp64] {over}")
    g = det_system(md, w, s)
    g.forces("edge_det")
    out = g.get_state()
    F, T, _, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, patchy_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, patchy_params(w))
    assert np.abs(T).max() > 0
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10


def test_bitwise_repeatable(md):
    """The same forces bit for bit on every call and in a second system; the
    same trajectory bit for bit over 60 steps (with list rebuilds)."""
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 7)
    say("[edge_det bitwise] lj4096")
    a = det_system(md, w, s)
    b = det_system(md, w, s)
    a.forces("edge_det")
    f0 = a.get_state()["f"]
    for _ in range(3):
        a.forces("edge_det")
        assert np.array_equal(a.get_state()["f"], f0)
    b.forces("edge_det")
    assert np.array_equal(b.get_state()["f"], f0)
    a.step(60, "edge_det")
    b.step(60, "edge_det")
    sa, sb = a.get_state(), b.get_state()
    assert a.stats()["rebuilds"] >= 2
    for key in ("x", "v", "f"):
        assert np.array_equal(sa[key], sb[key]), key


def test_patchy_bitwise_repeatable(md):
    w = WORKLOADS["patchy"].with_(n=3000)
    s = accepted_state(w, 8)
    say("[edge_det patchy bitwise]")
    a = det_system(md, w, s)
    b = det_system(md, w, s)
    a.step(30, "edge_det")
    b.step(30, "edge_det")
    sa, sb = a.get_state(), b.get_state()
    for key in ("x", "v", "f", "q", "angmom", "torque"):
        assert np.array_equal(sa[key], sb[key]), key


def test_trajectory_100_steps(md):
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 5)
    say("[edge_det trajectory] lj4096 100 steps")
    ref = oracle.run(s.x, s.v, s.box, pot="lj", nsteps=100, dt=w.dt, skin=w.skin,
                     lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    g = det_system(md, w, s)
    g.step(100, "edge_det")
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(out["v"] - ref["v"]).max() < 1e-9
    if ref["disp_margin"] > 1e-12:
        assert g.stats()["rebuilds"] == len(ref["rebuild_steps"])


def test_equals_vertex_and_atomic_edge(md):
    w = WORKLOADS["lj_small"].with_(n=5000)
    s = accepted_state(w, 6)
    say("[edge_det = vertex = edge]")
    g = det_system(md, w, s)
    _, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_abs=True)
    g.forces("edge_det")
    fd = g.get_state()["f"]
    g.forces("vertex")
    assert cond_rel_err(g.get_state()["f"], fd, A) <= 1e-10
    g.forces("edge")
    assert cond_rel_err(g.get_state()["f"], fd, A) <= 1e-10
    g.forces("edge_det")
    assert np.array_equal(g.get_state()["f"], fd)


def test_needs_edge_store(md):
    w = WORKLOADS["lj_small"].with_(n=500)
    s = accepted_state(w, 1)
    g = md.System(md.make_params(w))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    with pytest.raises(md.MDError) as ei:
        g.forces("edge_det")
    assert ei.value.status == -1
