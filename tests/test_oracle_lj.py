"""Pins of the FP64 oracle, Lennard-Jones part, against what the paper and the
mathematics fix (no GPU).  Each test names the property it pins and a plausible
oracle mistake it would catch."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS, make_state

from _helpers import accepted_state

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lj_closed_forms.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, rc, r, qty, val = line.split()
        rows.append((name, float(rc), float(r), qty, float(val)))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r[0]}-{r[1]}")
def test_lj_closed_forms(row):
    """Eq. (1) evaluated at exact rationals (catches a wrong prefactor,
    exponent, or a missing/extra shift)."""
    name, rc, r, qty, val = row
    if qty == "V":
        v, _ = oracle.lj_pair(r * r, oracle.LJ(rcut=1e6))  # V(1e6) ~ 1e-36
        assert v == pytest.approx(val, rel=1e-12, abs=1e-15)
        v0, _ = oracle.lj_pair(rc * rc, oracle.LJ(rcut=rc))
        assert v0 == 0.0  # shifted to zero exactly at the cut-off
    elif qty == "Vts":
        v, _ = oracle.lj_pair(r * r, oracle.LJ(rcut=rc))
        assert v == pytest.approx(val, rel=1e-12)
    elif qty == "-dV/dr":
        _, fs = oracle.lj_pair(r * r, oracle.LJ(rcut=rc))
        assert fs * r == pytest.approx(val, rel=1e-12)


def test_lj_minimum_and_zero_force():
    """The minimum of Eq. (1) is -eps at 2^(1/6) sigma, with zero force; force is
    repulsive inside and attractive outside (catches a sign error)."""
    p = oracle.LJ(eps=1.7, sigma=1.3, rcut=2.5 * 1.3)
    rmin = 2 ** (1 / 6) * p.sigma
    v, fs = oracle.lj_pair(rmin ** 2, p)
    vshift, _ = oracle.lj_pair(p.rcut ** 2, oracle.LJ(eps=p.eps, sigma=p.sigma, rcut=1e6))
    assert v + vshift == pytest.approx(-p.eps, rel=1e-13)
    assert abs(fs) < 1e-12
    _, f_in = oracle.lj_pair((0.95 * rmin) ** 2, p)
    _, f_out = oracle.lj_pair((1.05 * rmin) ** 2, p)
    assert f_in > 0 and f_out < 0  # force on j along x_j - x_i: pushes apart inside


def test_min_image():
    L = 10.0
    assert oracle.min_image(6.0, L) == pytest.approx(-4.0)
    assert oracle.min_image(-6.0, L) == pytest.approx(4.0)
    assert oracle.min_image(4.0, L) == pytest.approx(4.0)
    assert oracle.min_image(19.0, L) == pytest.approx(-1.0)


def test_two_particles_across_boundary():
    """A pair split by the periodic boundary interacts through the minimum
    image, with equal and opposite forces along the separation."""
    L = 8.0
    x = np.array([[0.2, 4.0, 4.0], [L - 0.9, 4.0, 4.0]])  # separation 1.1 across x=0
    F, e, w = oracle.lj_forces(x, L, oracle.LJ(), use_cells=False)
    v, fs = oracle.lj_pair(1.1 ** 2, oracle.LJ())
    # particle 1 sits at -1.1 in x relative to particle 0
    assert F[1, 0] == pytest.approx(fs * -1.1, rel=1e-13)
    assert F[0, 0] == pytest.approx(-F[1, 0], rel=1e-13)
    assert np.all(F[:, 1:] == 0)
    assert e.sum() == pytest.approx(v, rel=1e-13)


def _small_fluid(n=500, rho=0.8, seed=3):
    w = WORKLOADS["lj_small"].with_(n=n, rho=rho)
    return w, accepted_state(w, seed)


def test_newton_third_law():
    """Sum of all forces vanishes (Newton's third law, which the edge method
    relies on; catches a term added to one particle only)."""
    w, s = _small_fluid()
    F, _, _, A = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_abs=True)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * A.sum()


def test_forces_are_minus_gradient():
    """F = -grad E_pot by central differences (catches wrong derivative,
    sign, or a force/energy mismatch)."""
    w, s = _small_fluid(n=300, rho=0.9, seed=5)
    p = oracle.LJ()
    F, _, _ = oracle.lj_forces(s.x, s.box, p)
    rng = np.random.default_rng(0)
    h = 1e-5
    for i in rng.choice(s.x.shape[0], 8, replace=False):
        for c in range(3):
            xp, xm = s.x.copy(), s.x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            ep = oracle.lj_forces(xp, s.box, p)[1].sum()
            em = oracle.lj_forces(xm, s.box, p)[1].sum()
            fd = -(ep - em) / (2 * h)
            assert fd == pytest.approx(F[i, c], rel=1e-6, abs=1e-7)


def test_brute_force_equals_cells():
    """O(N^2) definition equals the cell-list enumeration, for pairs and forces."""
    w, s = _small_fluid(n=1500, rho=0.8, seed=7)
    rv = w.rcut + w.skin
    pb = oracle.pairs(s.x, s.box, rv, method="brute")
    pc = oracle.pairs(s.x, s.box, rv, method="cells")
    assert np.array_equal(pb, pc)
    Fb, eb, wb = oracle.lj_forces(s.x, s.box, oracle.LJ(), use_cells=False)
    Fc, ec, wc = oracle.lj_forces(s.x, s.box, oracle.LJ(), use_cells=True)
    np.testing.assert_allclose(Fc, Fb, rtol=0, atol=1e-11)
    np.testing.assert_allclose(ec, eb, rtol=0, atol=1e-12)


def test_pairs_match_distances_and_neighbors_of():
    """Pair set is exactly {i<j: r < r_v}; per-particle lists agree with it."""
    w, s = _small_fluid(n=400, rho=0.8, seed=11)
    rv = w.rcut + w.skin
    P = oracle.pairs(s.x, s.box, rv)
    d = s.x[:, None, :] - s.x[None, :, :]
    d -= s.box * np.rint(d / s.box)
    r = np.sqrt((d * d).sum(-1))
    iu = np.triu_indices(s.x.shape[0], 1)
    expect = np.stack(iu, axis=1)[r[iu] < rv]
    assert np.array_equal(P, expect.astype(np.int32))
    for i in (0, 17, 399):
        nb = oracle.neighbors_of(i, s.x, s.box, rv)
        ref = np.sort(np.concatenate([P[P[:, 0] == i, 1], P[P[:, 1] == i, 0]]))
        assert np.array_equal(nb, ref)


def test_force_one_matches_all():
    w, s = _small_fluid(n=300, seed=13)
    F, e, _ = oracle.lj_forces(s.x, s.box, oracle.LJ())
    for i in (0, 100, 299):
        f, ei = oracle.lj_force_one(i, s.x, s.box, oracle.LJ())
        np.testing.assert_allclose(f, F[i], atol=1e-12)
        assert ei == pytest.approx(e[i], abs=1e-13)


def test_virial_pair():
    """Per-particle virial halves r_ij . F_j of each pair: for two particles at
    distance r the total is r * (-dV/dr)."""
    L = 20.0
    r = 1.3
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    _, _, wv = oracle.lj_forces(x, L, oracle.LJ(), use_cells=False)
    _, fs = oracle.lj_pair(r * r, oracle.LJ())
    assert wv.sum() == pytest.approx(fs * r * r, rel=1e-13)


def test_energy_scale_pair_and_bound():
    """The per-particle energy scale: for two particles at distance r it sums,
    over both ends, to |4 (1/r)^12| + |4 (1/r)^6| + |V(rc)| (eps = sigma = 1),
    and on a fluid it bounds |e_i| (triangle inequality over the terms)."""
    L = 20.0
    r = 1.3
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    _, e, _, ea = oracle.lj_forces(x, L, oracle.LJ(), use_cells=False, with_eabs=True)
    vrc = 4.0 * (2.5 ** -12 - 2.5 ** -6)
    want = 4.0 * r ** -12 + 4.0 * r ** -6 + abs(vrc)
    assert ea.sum() == pytest.approx(want, rel=1e-14)
    assert ea[0] == pytest.approx(ea[1], rel=1e-15)
    w, s = _small_fluid(n=500, seed=21)
    _, e, _, ea = oracle.lj_forces(s.x, s.box, oracle.LJ(), with_eabs=True)
    assert (ea >= np.abs(e) - 1e-15).all()
    assert (ea > 0).all()


def _run(s, w, nsteps, dt):
    return oracle.run(s.x, s.v, s.box, pot="lj", nsteps=nsteps, dt=dt, skin=w.skin,
                      lj=oracle.LJ(w.eps, w.sigma, w.rcut))


def test_energy_conservation_and_dt2_scaling():
    """Velocity Verlet conserves energy with fluctuations scaling as dt^2
    (catches a wrong half-kick or a force/energy inconsistency)."""
    w, s = _small_fluid(n=256, rho=0.8, seed=17)
    out1 = _run(s, w, 200, 0.002)
    out2 = _run(s, w, 400, 0.001)
    e1 = out1["energies"][:, 0] + out1["energies"][:, 1]
    e2 = out2["energies"][:, 0] + out2["energies"][:, 1]
    f1 = e1.std()
    f2 = e2[::2].std()
    assert abs(e1[-1] - e1[0]) / 256 < 2e-4
    assert 2.5 < f1 / f2 < 6.0  # ~4 for a second-order integrator
    mom = out1["v"].sum(axis=0)
    assert np.abs(mom).max() < 1e-10


def test_time_reversibility():
    """Run N steps, negate v, run N steps: positions come back (velocity Verlet
    is time-reversible; catches an asymmetric update order)."""
    w, s = _small_fluid(n=200, rho=0.8, seed=19)
    fwd = _run(s, w, 50, 0.001)
    class S2:  # noqa: D401 - a tiny state holder
        pass
    s2 = S2()
    s2.x, s2.v, s2.box = fwd["x"], -fwd["v"], s.box
    back = _run(s2, w, 50, 0.001)
    d = back["x"] - s.x
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-back["v"], s.v, atol=1e-9)


def test_rebuild_schedule():
    """The list is built at t=0 and rebuilt only when the largest displacement
    since the last build exceeds half the skin."""
    w, s = _small_fluid(n=256, rho=0.8, seed=23)
    out = _run(s, w, 300, 0.002)
    rb = out["rebuild_steps"]
    assert rb[0] == 0 and len(rb) >= 2
    assert np.all(np.diff(rb) > 0)
    # velocities ~ sqrt(3T) ~ 2: half a skin (0.15) takes >= 0.15/vmax ~ 0.02 time units
    assert np.diff(rb).min() * 0.002 > 0.01


def test_rebuild_rule_reconstructed():
    """Rebuild steps equal those recomputed in numpy from the step-by-step
    trajectory: rebuild when max_i |x_i - x_i(last build)| > skin/2."""
    w, s = _small_fluid(n=216, rho=0.8, seed=29)
    nsteps, dt = 120, 0.002
    full = _run(s, w, nsteps, dt)

    class St:
        pass
    cur = St()
    cur.x, cur.v, cur.box = s.x.copy(), s.v.copy(), s.box
    traj = [cur.x.copy()]
    for _ in range(nsteps):  # chaining single steps reproduces the run exactly
        o = _run(cur, w, 1, dt)
        cur.x, cur.v = o["x"], o["v"]
        traj.append(cur.x.copy())
    np.testing.assert_array_equal(traj[-1], full["x"])
    expect, xb = [0], traj[0]
    for k in range(1, nsteps + 1):
        d = traj[k] - xb
        d -= s.box * np.rint(d / s.box)
        if np.sqrt((d * d).sum(1)).max() > w.skin / 2:
            expect.append(k)
            xb = traj[k]
    assert list(full["rebuild_steps"]) == expect
    assert len(expect) >= 3


def test_generator_margin_helper():
    """accepted_state keeps every pair distance 1e-9 away from r_c and r_v."""
    w = WORKLOADS["lj_small"]
    s = accepted_state(w, 1)
    m = oracle.pair_margin(s.x, s.box, [w.rcut, w.rcut + w.skin])
    assert m > 1e-9
    assert s.x.shape == (4096, 3)
