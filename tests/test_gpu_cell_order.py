"""GPU parity of the cell orders of the locality study: with the cells (and
so the slots) in row-major order without LDS staging, in Morton order and
along a Hilbert curve, the neighbour sets are the oracle's and the forces and
100-step trajectories match it, for both decompositions."""
import sys

import numpy as np
import pytest

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS

from _helpers import accepted_state, cond_rel_err

pytestmark = pytest.mark.gpu

ORDERS = ["row_major_gather", "morton", "hilbert"]


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import md as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def system(md, w, s, order):
    g = md.System(md.make_params(w, cell_order=order))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    return g


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("case", [("lj_small", {}), ("lj_small", {"n": 300}),
                                  ("lj_small", {"n": 5000})])
def test_lj(md, order, case):
    name, over = case
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 11)
    say(f"[cell order] {order} lj n={w.n}")
    g = system(md, w, s, order)
    assert g.stats()["tiles_staged"] == 0
    assert np.array_equal(g.pairs(), oracle.pairs(s.x, s.box, w.rv))
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
    for mode in ("vertex", "edge"):
        g.forces(mode)
        assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-10, mode


@pytest.mark.parametrize("order", ORDERS)
def test_patchy(md, order):
    w = WORKLOADS["patchy"].with_(n=3000)
    s = accepted_state(w, 12)
    say(f"[cell order] {order} patchy")
    g = system(md, w, s, order)
    assert np.array_equal(g.pairs(), oracle.pairs(s.x, s.box, w.rv))
    p = oracle.Patchy(eps=w.eps, sigma=w.sigma, rcut=w.rcut, eps_p=w.eps_p, w=w.patch_w,
                      delta=w.patch_delta, rpc=w.patch_rcut)
    F, T, _, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, p, with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, p)
    g.forces("vertex")
    out = g.get_state()
    assert cond_rel_err(out["f"], F, FP) <= 1e-10
    assert cond_rel_err(out["torque"], T, TP) <= 1e-10


@pytest.mark.parametrize("order", ORDERS)
def test_trajectory(md, order):
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 5)
    say(f"[cell order] {order} trajectory")
    ref = oracle.run(s.x, s.v, s.box, pot="lj", nsteps=100, dt=w.dt, skin=w.skin,
                     lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    g = system(md, w, s, order)
    g.step(100, "vertex")
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(out["v"] - ref["v"]).max() < 1e-9
