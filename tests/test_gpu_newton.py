"""GPU parity of the vertex pass with Newton's third law (LJ): each pair
evaluated once from the half list, the partner share added atomically into
m replicated force arrays (m >= 1, as the paper describes) or into a
per-workgroup LDS accumulator (m = 0).  Same bars as the other modes: FP64
forces within 1e-10 of the sum of the term magnitudes per component, FP32
pair maths within 1e-5, 100 steps within 1e-9 of the oracle."""
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


def system(md, w, s, prec="fp64", m=0):
    g = md.System(md.make_params(w, prec, newton_m=m))
    g.set_state(s.x, s.v)
    g.build()
    return g


CASES = {
    "lj20000_staged": ("lj_small", {"n": 20000}),
    "lj4096": ("lj_small", {}),
    "lj1000_ragged": ("lj_small", {"n": 1000}),
    "lj300_two_cells": ("lj_small", {"n": 300}),
    "lj_dilute": ("lj_small", {"n": 2000, "rho": 0.1}),
    "lj_dense_rc3": ("lj_many_dense", {"n": 30000}),
}


@pytest.mark.parametrize("m", [0, 1, 4, 16])
@pytest.mark.parametrize("case", list(CASES))
def test_newton_forces_fp64(md, case, m):
    name, over = CASES[case]
    w = WORKLOADS[name].with_(**over)
    s = accepted_state(w, 12)
    say(f"[newton fp64] {case} m={m}")
    g = system(md, w, s, m=m)
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
    for _ in range(2):  # the replicas are cleared by each pass
        g.forces("newton")
        assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-10


@pytest.mark.parametrize("m", [0, 8])
def test_newton_forces_fp32(md, m):
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 4)
    say(f"[newton fp32] m={m}")
    g = system(md, w, s, prec="fp32", m=m)
    g.forces("newton")
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_abs=True)
    assert cond_rel_err(g.get_state()["f"], F, A) <= 1e-5


@pytest.mark.parametrize("m", [0, 8])
def test_newton_trajectory_100_steps(md, m):
    w = WORKLOADS["lj_small"].with_(n=3000)
    s = accepted_state(w, 5)
    say(f"[newton trajectory] m={m}")
    ref = oracle.run(s.x, s.v, s.box, pot="lj", nsteps=100, dt=w.dt, skin=w.skin,
                     lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    g = system(md, w, s, m=m)
    g.step(100, "newton")
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(out["v"] - ref["v"]).max() < 1e-9
    if ref["disp_margin"] > 1e-12:
        assert g.stats()["rebuilds"] == len(ref["rebuild_steps"])


def test_newton_rejected_for_patchy(md):
    w = WORKLOADS["patchy"].with_(n=500)
    s = accepted_state(w, 1)
    g = md.System(md.make_params(w))
    g.set_state(s.x, s.v, s.q, s.angmom)
    g.build()
    with pytest.raises(md.MDError) as e:
        g.forces("newton")
    assert e.value.status == -1
