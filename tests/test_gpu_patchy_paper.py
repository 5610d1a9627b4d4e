"""GPU parity, the paper's patchy model (two polar patches, (sigma/r)^200 core,
patch range 0.18 sigma; Eqs. 2-4 with M = 2): forces, torques, energies,
neighbour sets and rotational velocity-Verlet trajectories of the HIP path
(through the C ABI) against the FP64 oracle, at the paper's three densities.

The inputs are chains of mostly aligned particles, so that a good share of the
patch pairs is bonded.  Bars as for the four-patch model: neighbour set
bit-exact; FP64 forces and torques within 1e-10 of the per-pair scale
sum_j |F_i(ij)| per component (and so of the larger per-term scale); FP32
patch terms within 1e-5 of the per-term scale (the error against the per-pair
scale is printed); 100 steps within 1e-9."""
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


def paper_params(w):
    assert w.patch_model == "polar2"
    return oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                         delta=w.patch_delta, rpc=w.patch_rcut, model=1)


def gpu_system(md, w, s, prec="fp64", edge_store=False):
    g = md.System(md.make_params(w, prec, edge_store=edge_store))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    return g


CASES = {
    "rho05_n3000": {"n": 3000},                    # 11 cells per side
    "rho03_n2000": {"n": 2000, "rho": 0.3},
    "rho01_n1500": {"n": 1500, "rho": 0.1},
    "rho05_small_box": {"n": 250},                 # 4 cells per side
    "rho05_ragged": {"n": 1001},
}


@pytest.mark.parametrize("case", list(CASES))
def test_neighbors_exact(md, case):
    w = WORKLOADS["patchy_paper"].with_(**CASES[case])
    s = accepted_state(w, 1)
    say(f"[patchy_paper neighbors] {case}")
    g = gpu_system(md, w, s)
    assert np.array_equal(g.pairs(), oracle.pairs(s.x, s.box, w.rv))


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode", ["vertex", "edge", "edge_det"])
def test_forces_torques_fp64(md, case, mode):
    w = WORKLOADS["patchy_paper"].with_(**CASES[case])
    s = accepted_state(w, 2)
    say(f"[patchy_paper fp64] {case} {mode}")
    g = gpu_system(md, w, s, edge_store=(mode == "edge_det"))
    g.forces(mode)
    out = g.get_state()
    F, T, e, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, paper_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, paper_params(w))
    assert e.sum() < -0.02 * w.n  # bonds formed
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10
    ke, pe, _ = g.energy()
    assert pe == pytest.approx(e.sum(), rel=0, abs=1e-12 * np.abs(e).sum())
    ep = g.particle_energies()
    np.testing.assert_allclose(ep, e, rtol=0, atol=1e-12 * np.abs(e).max())


@pytest.mark.parametrize("prec", ["fp32", "fp32_kahan"])
@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_forces_fp32(md, prec, mode):
    w = WORKLOADS["patchy_paper"].with_(n=3000)
    s = accepted_state(w, 3)
    say(f"[patchy_paper {prec}] {mode}")
    g = gpu_system(md, w, s, prec=prec)
    g.forces(mode)
    out = g.get_state()
    F, T, e, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, paper_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, paper_params(w))
    # bar: 1e-5 of the per-term scale (rounding of each term is what an FP32
    # evaluation adds); the error against the per-pair scale is reported
    say(f"[patchy_paper {prec} errors] {mode} per-term F %.2e T %.2e, per-pair F %.2e T %.2e" % (
        cond_rel_err(out["f"], F, FA), cond_rel_err(out["torque"], T, TA),
        cond_rel_err(out["f"], F, FP), cond_rel_err(out["torque"], T, TP)))
    assert cond_rel_err(out["f"], F, FA) <= 1e-5
    assert cond_rel_err(out["torque"], T, TA) <= 1e-5
    np.testing.assert_allclose(g.particle_energies(), e, rtol=0, atol=1e-6 * np.abs(e).max())


@pytest.mark.parametrize("mode", ["vertex", "edge", "edge_det"])
def test_trajectory_100_steps(md, mode):
    """Rotational velocity Verlet, 100 steps at dt = 0.001, against the oracle."""
    w = WORKLOADS["patchy_paper"].with_(n=2000)
    s = accepted_state(w, 5)
    say(f"[patchy_paper trajectory] {mode}")
    ref = oracle.run(s.x, s.v, s.box, pot="patchy", nsteps=100, dt=w.dt, skin=w.skin,
                     patchy=paper_params(w), q=s.q, angmom=s.angmom, inertia=w.inertia)
    g = gpu_system(md, w, s, edge_store=(mode == "edge_det"))
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


def test_full_size(md):
    """The full 131 072-particle system at rho = 0.5 (the bench workload),
    every particle, both decompositions."""
    w = WORKLOADS["patchy_paper"]
    s = accepted_state(w, 0)
    say("[patchy_paper full size] n=131072")
    F, T, e, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, paper_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, paper_params(w))
    g = gpu_system(md, w, s)
    for mode in ("vertex", "edge"):
        g.forces(mode)
        out = g.get_state()
        assert cond_rel_err(out["f"], F, FP) <= 1e-10, mode
        assert cond_rel_err(out["torque"], T, TP) <= 1e-10, mode


@pytest.mark.parametrize("n", [65536, 65537])
def test_vertex_lane_count_boundary(md, n):
    """The vertex pass runs four lanes per particle up to 65 536 particles and
    one lane above: both sides of the switch against the oracle, with energies."""
    w = WORKLOADS["patchy_paper"].with_(n=n)
    s = accepted_state(w, 4)
    say(f"[patchy_paper vertex lanes] n={n}")
    g = gpu_system(md, w, s)
    g.forces("vertex")
    out = g.get_state()
    F, T, e, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, paper_params(w), with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, paper_params(w))
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10
    np.testing.assert_allclose(g.particle_energies(), e, rtol=0, atol=1e-12 * np.abs(e).max())
