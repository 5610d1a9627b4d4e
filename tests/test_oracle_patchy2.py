"""Pins of the FP64 oracle, the paper's two-patch model (no GPU).

Model (Eqs. 2-4, M = 2, reading stated in oracle/oracle.c): core
(sigma/r)^200, patch attraction -eps_p exp(-1/2 (s/0.12 sigma)^10) between
patch points a distance delta from the centres on the body z axis, cut at
s = 0.18 sigma.  Pinned against a two-body closed form, finite differences of
the energy for forces and torques, Newton's third law, angular-momentum
balance, brute force vs cell list, the size of the truncation jump and energy
conservation of rotational velocity Verlet."""
import math

import numpy as np
import pytest

import oracle

P = oracle.Patchy.paper()
# rotation by 90 degrees about y: body z -> +x
QX = np.array([math.cos(math.pi / 4), 0.0, math.sin(math.pi / 4), 0.0])


@pytest.mark.parametrize("r", [0.98, 1.0, 1.03, 1.08, 1.12, 1.17, 1.179])
def test_two_body_closed_form(r):
    """Both particles with body z along +x, particle j at (r, 0, 0): the patch
    of i at +delta x faces the patch of j at -delta x (s = r - 2 delta), the
    other patch pairs are beyond 0.18: V = r^-200 - eps_p exp(-1/2 (s/w)^10),
    force along x, no torque."""
    L = 20.0
    xi = np.array([5.0, 5.0, 5.0])
    xj = xi + [r, 0, 0]
    V, Fj, ti, tj = oracle.patchy_pair(xi, xj, QX, QX, L, P)
    s = r - 2 * P.delta
    E = math.exp(-0.5 * (s / P.w) ** 10) if abs(s) < P.rpc else 0.0
    # (s/w)^10 amplifies the rounding of s tenfold, exp by the argument (<= 29)
    assert V == pytest.approx(r ** -200 - P.eps_p * E, rel=1e-11, abs=1e-300)
    dV = -200 * r ** -201 + (5 * P.eps_p * E * (s / P.w) ** 8 * s / P.w ** 2 if E else 0.0)
    assert Fj[0] == pytest.approx(-dV, rel=1e-11, abs=1e-13)
    # off-axis parts are rounding of the rotation matrix (1e-16) times the
    # pair stiffness
    tol = 1e-13 * max(1.0, abs(Fj[0]))
    assert abs(Fj[1]) < tol and abs(Fj[2]) < tol
    assert np.abs(ti).max() < tol and np.abs(tj).max() < tol


def test_bond_energy_and_truncation():
    """A touching bond (s = 0) is worth -eps_p; at the patch range the term is
    eps_p exp(-1/2 1.5^10) = 3.0e-13 eps_p, and zero beyond."""
    L = 20.0
    x0 = np.array([5.0, 5.0, 5.0])
    V, *_ = oracle.patchy_pair(x0, x0 + [1.0, 0, 0], QX, QX, L, P)
    assert V == pytest.approx(1.0 - 1.0, abs=1e-15)  # core 1 at r = sigma, bond -1
    jump = math.exp(-0.5 * 1.5 ** 10)
    assert 2.9e-13 < jump < 3.1e-13
    Vin, *_ = oracle.patchy_pair(x0, x0 + [1.18 - 1e-12, 0, 0], QX, QX, L, P)
    Vout, *_ = oracle.patchy_pair(x0, x0 + [1.18 + 1e-9, 0, 0], QX, QX, L, P)
    assert Vout == 0.0
    assert Vin == pytest.approx(1.18 ** -200 - jump, rel=1e-6)


def _rotate(q, axis, h):
    rq = np.array([math.cos(h / 2), *(math.sin(h / 2) * np.eye(3)[axis])])
    w1, x1, y1, z1 = rq
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _bonded_chain(n, seed):
    """A chain along x of particles whose z axes point along x, patches
    nearly in contact, with random tilts and offsets so that forces and
    torques are generic."""
    rng = np.random.default_rng(seed)
    x = np.zeros((n, 3))
    q = np.zeros((n, 4))
    for k in range(n):
        x[k] = [3.0 + 1.06 * k, 4.0, 4.0] + rng.uniform(-0.03, 0.03, 3)
        qk = QX.copy()
        for ax in range(3):
            qk = _rotate(qk, ax, rng.uniform(-0.12, 0.12))
        q[k] = qk / np.linalg.norm(qk)
    return x, q


def test_forces_and_torques_are_minus_gradient():
    box = 30.0
    x, q = _bonded_chain(8, 1)
    p = oracle.Patchy(**{**P.__dict__, "rpc": 0.0})  # untruncated: smooth surface
    F, T, e, _ = oracle.patchy_forces(x, q, box, p, use_cells=False)
    assert e.sum() < -1.0  # bonds formed
    assert np.abs(T).max() > 1e-3
    h = 1e-7
    for i in (0, 3, 7):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            ep = oracle.patchy_forces(xp, q, box, p, use_cells=False)[2].sum()
            em = oracle.patchy_forces(xm, q, box, p, use_cells=False)[2].sum()
            assert -(ep - em) / (2 * h) == pytest.approx(F[i, c], rel=1e-5, abs=1e-5)
            qp, qm = q.copy(), q.copy()
            qp[i] = _rotate(q[i], c, h)
            qm[i] = _rotate(q[i], c, -h)
            ep = oracle.patchy_forces(x, qp, box, p, use_cells=False)[2].sum()
            em = oracle.patchy_forces(x, qm, box, p, use_cells=False)[2].sum()
            assert -(ep - em) / (2 * h) == pytest.approx(T[i, c], rel=1e-5, abs=1e-5)


def test_pair_newton_and_angular_momentum():
    """Per pair, near-bonded orientations: tau_i + tau_j = r_ij x F_i."""
    rng = np.random.default_rng(4)
    box = 30.0
    hits = 0
    for _ in range(300):
        xi = rng.uniform(5, 6, 3)
        d = np.array([rng.uniform(1.0, 1.17), 0, 0]) + rng.uniform(-0.04, 0.04, 3)
        qi, qj = QX.copy(), QX.copy()
        for ax in range(3):
            qi = _rotate(qi, ax, rng.uniform(-0.2, 0.2))
            qj = _rotate(qj, ax, rng.uniform(-0.2, 0.2))
        V, Fj, ti, tj = oracle.patchy_pair(xi, xi + d, qi, qj, box, P)
        if np.abs(ti).max() > 1e-6:
            hits += 1
        scale = max(1.0, np.abs(Fj).max())
        np.testing.assert_allclose(ti + tj, np.cross(d, -Fj), atol=1e-12 * scale)
    assert hits > 100


def test_cells_equal_brute_force():
    rng = np.random.default_rng(7)
    n, box = 600, 11.0  # rho = 0.45
    x = rng.uniform(0, box, (n, 3))
    # keep centres apart (the core is stiff), then chain some pairs
    x[: n // 2] = x[: n // 2]
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    F, T, e, _, FA, _ = oracle.patchy_forces(x, q, box, P, use_cells=True, with_abs=True)
    F2, T2, e2, _ = oracle.patchy_forces(x, q, box, P, use_cells=False)
    np.testing.assert_allclose(F, F2, rtol=0, atol=1e-9 * max(FA.max(), 1.0))
    np.testing.assert_allclose(T, T2, rtol=0, atol=1e-9 * max(np.abs(T2).max(), 1.0))
    np.testing.assert_allclose(e, e2, rtol=1e-12, atol=1e-300)
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * FA.sum()


def test_rotational_velocity_verlet_energy_error_scales_dt2():
    """A bonded chain at low temperature: the largest total-energy excursion
    over a fixed time shrinks fourfold when dt halves (second order)."""
    x, q = _bonded_chain(12, 3)
    rng = np.random.default_rng(5)
    v = rng.normal(0, math.sqrt(0.15), (12, 3))
    v -= v.mean(0)
    L = rng.normal(0, math.sqrt(0.15), (12, 3))
    dev = []
    for dt, nsteps in ((0.0004, 100), (0.0002, 200)):
        out = oracle.run(x, v, 30.0, pot="patchy", nsteps=nsteps, dt=dt, skin=0.3, patchy=P,
                         q=q, angmom=L)
        E = out["energies"][:, 0] + out["energies"][:, 1]
        assert E[0] < 0
        dev.append(np.abs(E - E[0]).max())
    assert 3.0 < dev[0] / dev[1] < 5.0
