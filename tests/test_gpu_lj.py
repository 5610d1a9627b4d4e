"""GPU parity, Lennard-Jones: the HIP path (through the C ABI) against the FP64
oracle on the same seeded inputs.

Bars (written here, derived in the design notes):
  - neighbour pair set: bit-exact (sets compared in original ids);
  - FP64 forces: |F - F*| <= 1e-10 * sum_j |F*_ij| per component (the only
    differences are summation order and atomic order);
  - FP64 energies: per-particle |e - e*| <= 1e-12 * (1/2 sum_j |V*_ij|) and
    totals to 1e-12 relative to the sum of magnitudes;
  - FP32 pair maths: forces 1e-5 and per-particle energies 1e-6, each against
    the sum of the magnitudes of its terms (for V_ij: 4 eps (sigma/r)^12,
    4 eps (sigma/r)^6 and the shift);
  - 100 velocity-Verlet steps: positions and velocities within 1e-9, with the
    same number of list builds as the oracle's rebuild schedule.
"""
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


def gpu_system(md, w, s, prec="fp64"):
    sys_ = md.System(md.make_params(w, prec))
    sys_.set_state(s.x, s.v, s.q, s.angmom)
    sys_.build()
    return sys_


CASES = {
    # name: (workload, overrides) -- sizes span several tiles and ragged tails
    "lj4096": ("lj_small", {}),
    "lj1000_ragged": ("lj_small", {"n": 1000}),
    "lj5000_noncube": ("lj_small", {"n": 5000}),
    "lj300_two_cells": ("lj_small", {"n": 300}),          # 2 cells per side
    "lj170_min_box": ("lj_small", {"n": 170, "rho": 0.9}),   # box just above 2 r_v
    "lj_dense_rc3": ("lj_many_dense", {"n": 3000}),
    "lj_dilute": ("lj_small", {"n": 2000, "rho": 0.1}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_neighbor_set_exact(md, case):
    name, over = CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 1)
    say(f"[neighbors] {case} n={w.n} box={w.box:.4f}")
    g = gpu_system(md, w, s)
    got = g.pairs()
    ref = oracle.pairs(s.x, s.box, w.rv)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
    st = g.stats()
    assert st["pairs"] == len(ref)
    counts = np.bincount(ref.ravel(), minlength=w.n)
    assert st["max_list_len"] == counts.max()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_forces_fp64(md, case, mode):
    name, over = CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 2)
    say(f"[forces fp64] {case} {mode} n={w.n}")
    g = gpu_system(md, w, s)
    g.forces(mode)
    out = g.get_state()
    F, e, wv, A = oracle.lj_forces(s.x, s.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
    assert cond_rel_err(out["f"], F, A) <= 1e-10
    ke, pe, vir = g.energy()
    assert pe == pytest.approx(e.sum(), rel=0, abs=1e-12 * np.abs(e).sum() + 1e-300)
    assert vir == pytest.approx(wv.sum(), rel=0, abs=1e-12 * np.abs(wv).sum() + 1e-300)
    assert ke == pytest.approx(0.5 * w.mass * (s.v ** 2).sum(), rel=1e-13)
    ep = g.particle_energies()
    np.testing.assert_allclose(ep, e, rtol=0, atol=1e-12 * np.abs(e).max())


TILE_CASES = {
    "lj20000": ("lj_small", {"n": 20000}, "staged"),              # 10 cells per side
    "lj_dense_30000": ("lj_many_dense", {"n": 30000}, "staged"),  # 9 cells per side
    "lj_dilute": ("lj_small", {"n": 2000, "rho": 0.1}, "global"),
    "lj300_two_cells": ("lj_small", {"n": 300}, "global"),
}


@pytest.mark.parametrize("case", list(TILE_CASES))
def test_vertex_tile_paths(md, case):
    """Dense fluids stage most tiles' neighbour regions in LDS; dilute or tiny
    boxes fall back to global gathers; both give the oracle's forces."""
    name, over, expect = TILE_CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 9)
    say(f"[tiles] {case}")
    g = gpu_system(md, w, s)
    st = g.stats()
    if expect == "staged":  # small boxes: tiles spanning most of a row use gathers
        assert st["tiles_staged"] >= st["tiles_total"] // 2
    else:
        assert st["tiles_staged"] < st["tiles_total"]
    g.forces("vertex")
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
    assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-10


def test_vertex_equals_edge_many_calls(md):
    """Both decompositions give the same forces; repeated edge calls differ
    only at rounding level (atomic order)."""
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 3)
    say("[vertex=edge] lj4096")
    g = gpu_system(md, w, s)
    _, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_abs=True)
    g.forces("vertex")
    fv = g.get_state()["f"]
    g.forces("vertex")
    assert np.array_equal(fv, g.get_state()["f"])  # vertex is deterministic
    for _ in range(3):
        g.forces("edge")
        fe = g.get_state()["f"]
        assert cond_rel_err(fe, fv, A) <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "fp32_kahan"])
@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_forces_fp32(md, prec, mode):
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 4)
    say(f"[forces {prec}] {mode}")
    g = gpu_system(md, w, s, prec=prec)
    g.forces(mode)
    F, e, _, A, EA = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_abs=True, with_eabs=True)
    assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-5
    ep = g.particle_energies()
    assert cond_rel_err(ep, e, EA) <= 1e-6


@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_trajectory_100_steps(md, mode):
    """The small LJ workload: 100 velocity-Verlet steps at dt=0.001 with the
    device-side rebuild rule, against the oracle's run."""
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 5)
    say(f"[trajectory] lj4096 {mode} 100 steps")
    ref = oracle.run(s.x, s.v, s.box, pot="lj", nsteps=100, dt=w.dt, skin=w.skin,
                     lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    g = gpu_system(md, w, s)
    g.step(100, mode)
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(out["v"] - ref["v"]).max() < 1e-9
    st = g.stats()
    if ref["disp_margin"] > 1e-12:
        assert st["rebuilds"] == len(ref["rebuild_steps"])
    ke, pe, _ = g.energy()
    assert ke + pe == pytest.approx(ref["energies"][-1, 0] + ref["energies"][-1, 1], abs=1e-8)


def test_trajectory_with_rebuilds(md):
    """Longer run at a larger time step so the list is rebuilt many times."""
    w = WORKLOADS["lj_small"].with_(n=2000, dt=0.004)
    s = accepted_state(w, 6)
    say("[trajectory] lj2000 dt=0.004 150 steps vertex")
    ref = oracle.run(s.x, s.v, s.box, pot="lj", nsteps=150, dt=w.dt, skin=w.skin,
                     lj=oracle.LJ())
    g = gpu_system(md, w, s)
    g.step(150, "vertex")
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-8
    st = g.stats()
    assert len(ref["rebuild_steps"]) >= 4
    if ref["disp_margin"] > 1e-12:
        assert st["rebuilds"] == len(ref["rebuild_steps"])


@pytest.mark.parametrize("n,dt,steps", [(3000, 0.005, 90), (4096, 0.001, 60), (700, 0.006, 37)])
def test_fused_steps_equal_single_steps(md, n, dt, steps):
    """md_step(k) of the vertex LJ mode runs its fused launches in batches and
    enqueues a list rebuild when a launch reports one due (launches after it
    do nothing until the host resumes); k calls of md_step(1) run the
    per-step sequence (rebuild test chain, then forces).  The same arithmetic
    and the same rebuild steps give bitwise the same state -- at time steps
    that rebuild every few steps, so batches stop and resume many times."""
    w = WORKLOADS["lj_small"].with_(n=n, dt=dt)
    s = accepted_state(w, 8)
    say(f"[fused batches] lj n={n} dt={dt} {steps} steps")
    a = gpu_system(md, w, s)
    a.step(steps, "vertex")
    b = gpu_system(md, w, s)
    for _ in range(steps):
        b.step(1, "vertex")
    sa, sb = a.get_state(), b.get_state()
    ta, tb = a.stats(), b.stats()
    a.close()
    b.close()
    say(f"  list builds {ta['rebuilds']} / {tb['rebuilds']}")
    assert ta["rebuilds"] == tb["rebuilds"]
    if dt > 0.004:
        assert ta["rebuilds"] >= 5
    for key in ("x", "v", "f"):
        assert np.array_equal(sa[key], sb[key]), key


def test_overflow_is_reported(md):
    w = WORKLOADS["lj_small"].with_(max_neighbors=16)
    s = accepted_state(w, 7)
    say("[overflow] max_neighbors=16")
    g = gpu_system(md, w, s)
    with pytest.raises(md.MDError) as ei:
        g.step(1, "vertex")
    assert ei.value.status == -4


def test_nonfinite_is_reported(md):
    w = WORKLOADS["lj_small"].with_(n=500)
    s = accepted_state(w, 8)
    x = s.x.copy()
    x[1] = x[0]  # coincident particles: 1/r^2 overflows
    say("[nonfinite] coincident particles")
    g = md.System(md.make_params(w))
    g.set_state(x, s.v)
    g.build()
    with pytest.raises(md.MDError) as ei:
        g.step(1, "vertex")
    assert ei.value.status == -6


def test_call_order_errors(md):
    w = WORKLOADS["lj_small"].with_(n=500)
    g = md.System(md.make_params(w))
    with pytest.raises(md.MDError) as ei:
        g.forces("vertex")
    assert ei.value.status == -7
    with pytest.raises(md.MDError):
        g.build_neighbors()
    # between the cell sort and the list build the momenta sit in the reorder
    # buffers: a thermostat call there would be lost, so it is refused
    s = accepted_state(w, 9)
    g.set_state(s.x, s.v)
    g.build_cells()
    with pytest.raises(md.MDError) as ei:
        g.thermostat(1.0, 0.5, 1, 0)
    assert ei.value.status == -7
    g.build_neighbors()
    g.thermostat(1.0, 0.5, 1, 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonzero_pairs(md, prec):
    """md_stats' nonzero_pairs: the half-list pairs with a non-zero LJ force,
    i.e. those with r < r_c (the force vanishes exactly only at isolated
    distances no seeded pair hits), against the oracle's pair set at r_c."""
    w = WORKLOADS["lj_small"].with_(n=3000)
    s = accepted_state(w, 10)
    say(f"[nonzero pairs] {prec}")
    g = gpu_system(md, w, s, prec)
    st = g.stats()
    assert st["pairs"] == len(oracle.pairs(s.x, s.box, w.rv))
    assert st["nonzero_pairs"] == len(oracle.pairs(s.x, s.box, w.rcut))
