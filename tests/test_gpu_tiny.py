"""GPU parity at the smallest sizes the boundary accepts: two particles (one
partial tile), a tile minus one, one full tile and a tile plus one, in boxes of
two cells per side (just above twice the list range) and of three (the staged
region path), against the FP64 oracle.  Bars as in test_gpu_lj: the pair set
bit-exact, FP64 forces 1e-10 of the per-component sum of term magnitudes,
trajectories 1e-9 with the oracle's rebuild count."""
import sys

import numpy as np
import pytest

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS

from _helpers import cond_rel_err

pytestmark = pytest.mark.gpu

SIZES = [2, 3, 63, 64, 65]
BOXES = {"two_cells": 6.0, "three_cells": 8.7}  # 2 r_v = 5.6; 3 r_v = 8.4


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import md as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def workload(n, box):
    return WORKLOADS["lj_small"].with_(n=n, rho=n / box ** 3)


def tiny_state(w, seed):
    """Seeded positions with no pair closer than 0.95 sigma and no distance
    within 1e-6 of r_c or r_v; two particles sit 1.07 sigma apart across the
    periodic boundary in x.  Velocities Gaussian with the mean removed."""
    rng = np.random.default_rng(seed)
    L = w.box
    if w.n == 2:
        x = np.array([[0.3, 0.5 * L, 0.5 * L], [L - 0.75, 0.5 * L + 0.2, 0.5 * L - 0.1]])
    else:
        for _ in range(1000):
            x = np.zeros((0, 3))
            while len(x) < w.n:
                c = rng.uniform(0, L, 3)
                d = x - c
                d -= L * np.rint(d / L)
                if len(x) == 0 or np.min(np.sum(d * d, axis=1)) > 0.95 ** 2:
                    x = np.vstack([x, c])
            if oracle.pair_margin(x, L, [w.rcut, w.rcut + w.skin]) > 1e-6:
                break
    v = rng.normal(0.0, 1.0, (w.n, 3))
    v -= v.mean(axis=0)
    return x, v


def system(md, w, x, v):
    g = md.System(md.make_params(w, "fp64"))
    g.set_state(x, v)
    g.build()
    return g


@pytest.mark.parametrize("box", list(BOXES))
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_tiny_pairs_and_forces(md, n, box, mode):
    w = workload(n, BOXES[box])
    x, v = tiny_state(w, 11 + n)
    say(f"[tiny forces] n={n} {box} box={w.box:.3f} {mode}")
    g = system(md, w, x, v)
    ref = oracle.pairs(x, w.box, w.rv)
    got = g.pairs()
    assert got.shape == ref.shape and np.array_equal(got, ref)
    g.forces(mode)
    out = g.get_state()
    F, e, wv, A = oracle.lj_forces(x, w.box, oracle.LJ(w.eps, w.sigma, w.rcut), with_abs=True)
    if n == 2:
        assert np.abs(F).max() > 0  # the pair across the boundary interacts
    assert cond_rel_err(out["f"], F, A) <= 1e-10
    ke, pe, vir = g.energy()
    assert pe == pytest.approx(e.sum(), rel=0, abs=1e-12 * np.abs(e).sum() + 1e-300)
    assert vir == pytest.approx(wv.sum(), rel=0, abs=1e-12 * np.abs(wv).sum() + 1e-300)
    g.close()


@pytest.mark.parametrize("box", list(BOXES))
@pytest.mark.parametrize("n", [2, 65])
@pytest.mark.parametrize("mode", ["vertex", "edge"])
def test_tiny_trajectory(md, n, box, mode):
    """300 steps at dt = 0.004 (the fused vertex step and device-side
    rebuilds on a one- or two-tile system) against the oracle's run."""
    w = workload(n, BOXES[box]).with_(dt=0.004)
    x, v = tiny_state(w, 21 + n)
    say(f"[tiny trajectory] n={n} {box} {mode} 300 steps")
    ref = oracle.run(x, v, w.box, pot="lj", nsteps=300, dt=w.dt, skin=w.skin,
                     lj=oracle.LJ(w.eps, w.sigma, w.rcut))
    g = system(md, w, x, v)
    g.step(300, mode)
    out = g.get_state()
    d = out["x"] - ref["x"]
    d -= w.box * np.rint(d / w.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(out["v"] - ref["v"]).max() < 1e-9
    if ref["disp_margin"] > 1e-12:
        assert g.stats()["rebuilds"] == len(ref["rebuild_steps"])
    g.close()
