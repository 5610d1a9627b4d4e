"""GPU parity, patchy particles: forces, torques, energies, neighbour sets and
rotational velocity-Verlet trajectories of the HIP path (through the C ABI)
against the FP64 oracle on the same seeded inputs.

Bars as for LJ: neighbour set bit-exact; FP64 forces and torques within
1e-10 of the per-pair scale sum_j |F_i(ij)| per component (and so of the
larger per-term scale); FP32 pair maths within 1e-5 of the per-term scale (the
error against the per-pair scale is printed); 100 steps within 1e-9
(quaternions up to sign)."""
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


def patchy_params(w):
    return oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                         delta=w.patch_delta, rpc=w.patch_rcut)


def gpu_system(md, w, s, prec="fp64"):
    g = md.System(md.make_params(w, prec))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    return g


CASES = {
    "patchy3000": ("patchy", {"n": 3000}),                 # 10 cells per side
    "patchy_dense": ("patchy", {"n": 2000, "rho": 0.9}),   # many bonds and cores
    "patchy_small_box": ("patchy", {"n": 200, "rho": 0.5}),  # 3 cells per side
    "patchy_no_rpc": ("patchy", {"n": 1500, "patch_rcut": 0.0}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_patchy_neighbors_exact(md, case):
    name, over = CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 1)
    say(f"[patchy neighbors] {case}")
    g = gpu_system(md, w, s)
    assert np.array_equal(g.pairs(), oracle.pairs(s.x, s.box, w.rv))


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_patchy_forces_torques_fp64(md, case, mode):
    name, over = CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 2)
    say(f"[patchy fp64] {case} {mode}")
    g = gpu_system(md, w, s)
    g.forces(mode)
    out = g.get_state()
    F, T, e, wv, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, patchy_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, patchy_params(w))
    assert np.abs(T).max() > 0  # orientations matter in this configuration
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10
    ke, pe, vir = g.energy()
    assert pe == pytest.approx(e.sum(), rel=0, abs=1e-12 * np.abs(e).sum() + 1e-300)
    ekin = 0.5 * w.mass * (s.v ** 2).sum() + 0.5 * (s.angmom ** 2).sum() / w.inertia
    assert ke == pytest.approx(ekin, rel=1e-13)
    ep = g.particle_energies()
    np.testing.assert_allclose(ep, e, rtol=0, atol=1e-12 * max(np.abs(e).max(), 1e-300))


def test_patchy_edge_region_accumulation(md):
    """The four-patch edge pass sums a tile's partner and row shares in LDS
    over the tile's region (slot and image of each partner looked up at the
    half-list fill); tiles without a region add with global atomics.  Here a
    tile covers about 13 of a row's 16 cells, so most tiles span two rows of
    cells; the result is held to the FP64 bars."""
    w = WORKLOADS["patchy"].with_(n=20000, rho=0.7)
    s = accepted_state(w, 4)
    g = gpu_system(md, w, s)
    st = g.stats()
    say(f"[patchy edge regions] tiles with a region {st['tiles_staged']}/{st['tiles_total']}")
    assert 0 < st["tiles_staged"] <= st["tiles_total"]
    g.forces("edge")
    out = g.get_state()
    g.close()
    F, T, _, _, _, _ = oracle.patchy_forces(s.x, s.q, s.box, patchy_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, patchy_params(w))
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10


@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_patchy_forces_fp32(md, mode):
    w = WORKLOADS["patchy"].with_(n=3000)
    s = accepted_state(w, 3)
    say(f"[patchy fp32] {mode}")
    g = gpu_system(md, w, s, prec="fp32")
    g.forces(mode)
    out = g.get_state()
    F, T, e, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, patchy_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, patchy_params(w))
    # bar: 1e-5 of the per-term scale (rounding of each term is what an FP32
    # evaluation adds); the error against the per-pair scale is reported
    say(f"[patchy fp32 errors] {mode} per-term F %.2e T %.2e, per-pair F %.2e T %.2e" % (
        cond_rel_err(out["f"], F, FA), cond_rel_err(out["torque"], T, TA),
        cond_rel_err(out["f"], F, FP), cond_rel_err(out["torque"], T, TP)))
    assert cond_rel_err(out["f"], F, FA) <= 1e-5
    assert cond_rel_err(out["torque"], T, TA) <= 1e-5


@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_patchy_trajectory_100_steps(md, mode):
    """Rotational velocity Verlet, 100 steps at dt = 0.001, against the oracle."""
    w = WORKLOADS["patchy"].with_(n=2000)
    s = accepted_state(w, 5)
    say(f"[patchy trajectory] {mode}")
    ref = oracle.run(s.x, s.v, s.box, pot="patchy", nsteps=100, dt=w.dt, skin=w.skin,
                     patchy=patchy_params(w), q=s.q, angmom=s.angmom, inertia=w.inertia)
    g = gpu_system(md, w, s)
    g.step(100, mode)
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(out["v"] - ref["v"]).max() < 1e-9
    assert np.abs(out["angmom"] - ref["angmom"]).max() < 1e-9
    dots = np.abs((out["q"] * ref["q"]).sum(1))
    assert np.abs(dots - 1).max() < 1e-12
    if ref["disp_margin"] > 1e-12:
        assert g.stats()["rebuilds"] == len(ref["rebuild_steps"])


def test_patchy_vertex_equals_edge(md):
    w = WORKLOADS["patchy"].with_(n=3000)
    s = accepted_state(w, 6)
    g = gpu_system(md, w, s)
    _, _, _, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, patchy_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, patchy_params(w))
    g.forces("vertex")
    a = g.get_state()
    g.forces("edge")
    b = g.get_state()
    assert cond_rel_err(b["f"], a["f"], FP) <= 1e-10
    assert cond_rel_err(b["torque"], a["torque"], TP) <= 1e-10


@pytest.mark.parametrize("mode", ["edge", "edge_det"])
def test_sparse_half_list(md, mode):
    """A dilute random fluid (rho = 0.02, uniform positions, random
    orientations): about one pair per four particles, so a 64-entry chunk of
    the half list spans hundreds of rows -- the edge pass finds each entry's
    row by binary search there."""
    w = WORKLOADS["patchy"].with_(n=20000, rho=0.02)
    rng = np.random.default_rng(5)
    L = w.box
    x = rng.uniform(0.0, L, size=(w.n, 3))
    q = rng.normal(size=(w.n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    zero = np.zeros((w.n, 3))
    assert oracle.pair_margin(x, L, [w.rcut, w.rv]) > 1e-9
    say(f"[patchy sparse half list] {mode}")
    g = md.System(md.make_params(w, "fp64", edge_store=(mode == "edge_det")))
    g.set_state(x, zero, q, zero)
    g.build()
    st = g.stats()
    assert 0 < st["pairs"] < w.n // 2
    g.forces(mode)
    out = g.get_state()
    F, T, _, _, FA, TA = oracle.patchy_forces(x, q, L, patchy_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(x, q, L, patchy_params(w))
    assert np.count_nonzero(np.abs(T).sum(1)) > 100
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10


def test_patchy_nonzero_pairs(md):
    """md_stats' nonzero_pairs for patchy particles: half-list pairs whose
    force or either torque is non-zero, against the oracle's pair function
    evaluated on every listed pair."""
    w = WORKLOADS["patchy"].with_(n=1200)
    s = accepted_state(w, 21)
    say("[patchy nonzero pairs]")
    g = gpu_system(md, w, s)
    st = g.stats()
    pairs = oracle.pairs(s.x, s.box, w.rv)
    assert st["pairs"] == len(pairs)
    pp = patchy_params(w)
    nz = 0
    for i, j in pairs:
        _, fj, ti, tj = oracle.patchy_pair(s.x[i], s.x[j], s.q[i], s.q[j], s.box, pp)
        nz += bool(np.any(fj != 0) or np.any(ti != 0) or np.any(tj != 0))
    assert st["nonzero_pairs"] == nz
    assert 0 < nz < len(pairs)

