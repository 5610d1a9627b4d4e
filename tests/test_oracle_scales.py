"""Pins of the oracle's tolerance scales (no GPU).

Every force and torque parity bar divides |F - F*| by a per-component scale
that the oracle returns beside F*: for Lennard-Jones Fabs = sum_j |F_ij,c|;
for patchy particles Fabs / Tabs sum the magnitudes of the individual terms
of each pair (the core, and the Gaussian and the two cosine parts of every
patch pair), and or_patchy_pair_scales gives the per-pair sums
sum_j |F_i(ij),c|, sum_j |tau_i(ij),c|.  A wrong factor or term in these
scales would loosen or tighten every bar without any other test noticing, so
each is pinned here against a value fixed independently of the oracle's code:
a two-body closed form written out for the geometry, a numpy recomputation
from the oracle's single-pair routines, the triangle inequality, and a
measured bound on how far the per-term scale exceeds the per-pair one.
The generator's margin helper is pinned against a numpy brute force."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_1401_4350_amd.inputs import WORKLOADS, make_state

from _helpers import accepted_state

E0 = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
EZ = np.array([0.0, 0.0, 1.0])


def _quat(rot):
    x, y, z, w = rot.as_quat()
    return np.array([w, x, y, z])


def _pointing(body_axis, theta):
    """Quaternion that turns body_axis onto (cos theta, sin theta, 0)."""
    base, _ = Rotation.align_vectors([[1.0, 0.0, 0.0]], [body_axis])
    return _quat(Rotation.from_rotvec([0.0, 0.0, theta]) * base)


def _two_particles(r, q0, q1, L=20.0):
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    return x, np.stack([q0, q1]), L


# ---------------------------------------------------------------------------
# Lennard-Jones
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r", [0.9, 1.12, 1.5, 2.2, 2.49])
def test_lj_scale_of_one_pair(r):
    """Two particles along a general direction: Fabs of each equals |F| of
    that particle per component (one term per pair), and Eabs is half the sum
    of |4 eps (sigma/r)^12|, |4 eps (sigma/r)^6| and |V(r_c)| (Eq. 1)."""
    p = oracle.LJ(eps=1.3, sigma=1.1, rcut=2.5 * 1.1)
    d = np.array([0.48, -0.6, 0.64])  # unit vector
    x = np.array([[3.0, 4.0, 5.0], [3.0, 4.0, 5.0]])
    x[1] += r * d
    F, e, _, A, EA = oracle.lj_forces(x, 30.0, p, use_cells=False, with_abs=True,
                                      with_eabs=True)
    np.testing.assert_array_equal(A, np.abs(F))
    s6 = (p.sigma / r) ** 6
    src6 = (p.sigma / p.rcut) ** 6
    vrc = 4 * p.eps * (src6 * src6 - src6)
    ref = 0.5 * (4 * p.eps * s6 * s6 + 4 * p.eps * s6 + abs(vrc))
    np.testing.assert_allclose(EA, [ref, ref], rtol=1e-13)
    # and the force itself is the closed form 24 eps (2 s^12 - s^6) / r along d
    fmag = 24 * p.eps * (2 * s6 * s6 - s6) / r
    np.testing.assert_allclose(F[1], fmag * d, rtol=1e-12, atol=1e-15)


def test_lj_scale_equals_pair_sum():
    """On a 300-particle fluid, Fabs equals sum_j |F_ij,c| recomputed in numpy
    from or_lj_pair of every pair within r_c (minimum image), and
    |F| <= Fabs (triangle inequality).  Catches an extra factor, a dropped
    pair or a component mix-up in the scale."""
    w = WORKLOADS["lj_small"].with_(n=300)
    s = accepted_state(w, 3)
    p = oracle.LJ(w.eps, w.sigma, w.rcut)
    F, _, _, A = oracle.lj_forces(s.x, s.box, p, use_cells=False, with_abs=True)
    n = s.x.shape[0]
    ref = np.zeros((n, 3))
    for i in range(n):
        d = s.x - s.x[i]
        d -= s.box * np.rint(d / s.box)
        r2 = (d * d).sum(1)
        for j in np.nonzero((r2 < w.rcut ** 2) & (np.arange(n) != i))[0]:
            _, fs = oracle.lj_pair(float(r2[j]), p)
            ref[i] += np.abs(fs * d[j])
    np.testing.assert_allclose(A, ref, rtol=1e-13)
    assert np.all(np.abs(F) <= A * (1 + 1e-14))


# ---------------------------------------------------------------------------
# Patchy particles: one facing pair, patch of particle 0 tilted by theta
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("theta", [0.0, 0.15, -0.3])
@pytest.mark.parametrize("r", [0.98, 1.05, 1.12])
def test_tetra_term_scales_of_a_tilted_facing_pair(r, theta):
    """Four-patch model.  Particle 0's patch along u = (cos t, sin t, 0),
    particle 1 at (r, 0, 0) with a patch along -x; the other six patches are
    back-facing (checked), so one patch pair acts, with c_i = cos t, c_j = 1.
    With d = (r - delta (1 + cos t), -delta sin t, 0) and
    g = -eps_p exp(-|d|^2 / w^2), the term magnitudes of the force are
      Gaussian   2 |g| cos^2 t |d_c| / w^2
      cosine i   2 |g| cos t |(u - cos t x)_c| / r   (only y: sin t)
      cosine j   2 |g| cos^2 t |(x - x)_c| / r = 0
    plus the WCA core |24 eps (2 s^12 - s^6) / r| along x when r < 2^(1/6),
    and of the torque on particle 0 (z only)
      |u x (2 delta g cos^2 t d / w^2)| + |u x (2 g cos t x)|."""
    P = oracle.Patchy()
    q0 = _pointing(E0, theta)
    q1 = _pointing(E0, math.pi)
    x, q, L = _two_particles(r, q0, q1)
    u0 = oracle.quat_to_matrix(q0) @ (np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1],
                                                  [-1, -1, 1]]).T / math.sqrt(3))
    assert u0[0, 0] == pytest.approx(math.cos(theta)) and np.all(u0[0, 1:] < 0)
    F, T, _, _, FA, TA = oracle.patchy_forces(x, q, L, P, use_cells=False, with_abs=True)
    c, s = math.cos(theta), math.sin(theta)
    d = np.array([r - P.delta * (1 + c), -P.delta * s, 0.0])
    g = -P.eps_p * math.exp(-(d @ d) / P.w ** 2)
    G = g * c * c
    fa = 2 * abs(G) * np.abs(d) / P.w ** 2 + 2 * abs(g) * c * np.array([0.0, abs(s), 0.0]) / r
    if r * r < 2 ** (1 / 3):
        s6 = (P.sigma / r) ** 6
        fa[0] += abs(24 * P.eps * (2 * s6 * s6 - s6) / r)
    u = np.array([c, s, 0.0])
    ta = np.abs(np.cross(u, 2 * P.delta * G * d / P.w ** 2)) + np.abs(np.cross(u, [2 * g * c, 0, 0]))
    # components that vanish in the closed form carry the rounding of the
    # quaternion (an ulp of the pair's scale)
    tiny = 1e-12 * fa.max()
    np.testing.assert_allclose(FA[0], fa, rtol=1e-12, atol=tiny)
    np.testing.assert_allclose(TA[0], ta, rtol=1e-12, atol=tiny)
    # the per-pair scales of the same pair are the net magnitudes
    FP, TP = oracle.patchy_pair_scales(x, q, L, P, use_cells=False)
    np.testing.assert_array_equal(FP, np.abs(F))
    np.testing.assert_array_equal(TP, np.abs(T))
    assert np.all(FP <= FA * (1 + 1e-14)) and np.all(TP[0] <= TA[0] * (1 + 1e-14))


@pytest.mark.parametrize("theta", [0.0, 0.2, -0.25])
@pytest.mark.parametrize("r", [0.98, 1.02, 1.06])
def test_polar2_term_scales_of_a_tilted_facing_pair(r, theta):
    """Two-patch model.  Particle 0's axis along u = (cos t, sin t, 0) (patches
    at +-delta u), particle 1 at (r, 0, 0) with its axis along x; only the
    facing patch pair (+u, -x) is within the patch range, with
    d = (r - delta (1 + cos t), -delta sin t, 0), x = |d|^2 / w^2,
    E = exp(-x^5 / 2) and k = 5 eps_p E x^4 / w^2.  Term magnitudes of the
    force: the core 200 (sigma/r)^200 / r along x and |k d_c|; of the torque
    on particle 0: |u x (delta k d)| (z only)."""
    P = oracle.Patchy.paper()
    x, q, L = _two_particles(r, _pointing(EZ, theta), _pointing(EZ, 0.0))
    F, T, _, _, FA, TA = oracle.patchy_forces(x, q, L, P, use_cells=False, with_abs=True)
    c, s = math.cos(theta), math.sin(theta)
    d = np.array([r - P.delta * (1 + c), -P.delta * s, 0.0])
    assert math.sqrt(d @ d) < P.rpc
    xx = (d @ d) / P.w ** 2
    k = 5 * P.eps_p * math.exp(-0.5 * xx ** 5) * xx ** 4 / P.w ** 2
    fa = np.abs(k * d)
    fa[0] += 200 * (P.sigma / r) ** 200 / r
    u = np.array([c, s, 0.0])
    ta = np.abs(np.cross(u, P.delta * k * d))
    tiny = 1e-12 * fa.max()
    np.testing.assert_allclose(FA[0], fa, rtol=1e-12, atol=tiny)
    np.testing.assert_allclose(TA[0], ta, rtol=1e-12, atol=tiny)
    FP, TP = oracle.patchy_pair_scales(x, q, L, P, use_cells=False)
    np.testing.assert_array_equal(FP, np.abs(F))
    np.testing.assert_array_equal(TP, np.abs(T))


# ---------------------------------------------------------------------------
# Patchy particles: fluids
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("model", ["patchy", "patchy_paper"])
def test_patchy_pair_scales_equal_pair_sums(model):
    """or_patchy_pair_scales equals sum_j |F_j(ij)|, sum_j |tau_i(ij)| from
    or_patchy_pair over every pair of a small fluid (python loop), and the
    cell-list and brute-force enumerations agree."""
    w = WORKLOADS[model].with_(n=120)
    s = accepted_state(w, 2)
    p = oracle.Patchy() if model == "patchy" else oracle.Patchy.paper()
    n = s.x.shape[0]
    ref_f, ref_t = np.zeros((n, 3)), np.zeros((n, 3))
    for i in range(n):
        for j in range(n):
            if i != j:
                _, fj, ti, _ = oracle.patchy_pair(s.x[i], s.x[j], s.q[i], s.q[j], s.box, p)
                ref_f[i] += np.abs(fj)
                ref_t[i] += np.abs(ti)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, p, use_cells=False)
    np.testing.assert_allclose(FP, ref_f, rtol=1e-13, atol=0)
    np.testing.assert_allclose(TP, ref_t, rtol=1e-13, atol=0)
    FPc, TPc = oracle.patchy_pair_scales(s.x, s.q, s.box, p, use_cells=True)
    np.testing.assert_allclose(FPc, FP, rtol=1e-13, atol=0)
    np.testing.assert_allclose(TPc, TP, rtol=1e-13, atol=0)


# Bounds on per-term / per-pair, measured on 1 500-particle fluids of each
# model (seed 1): four patches median 1.003, 99th percentile 2.6, largest
# 27 (force); two patches median 1.000, 99th percentile 1.04; the sums over
# all components differ by 5 % and below 0.1 %.
RATIO_BOUNDS = {"patchy": dict(median=1.02, p99=4.0, total=1.10),
                "patchy_paper": dict(median=1.001, p99=1.2, total=1.01)}


@pytest.mark.parametrize("model", ["patchy", "patchy_paper"])
def test_term_scale_against_pair_scale(model):
    """|F| <= per-pair scale <= per-term scale on a 1 500-particle fluid (the
    triangle inequality, twice), and the per-term scale exceeds the per-pair
    one by no more than the stated bounds: the FP32 bar judged against the
    per-term scale is looser than the per-pair one by these factors."""
    w = WORKLOADS[model].with_(n=1500)
    s = accepted_state(w, 1)
    p = oracle.Patchy() if model == "patchy" else oracle.Patchy.paper()
    F, T, _, _, FA, TA = oracle.patchy_forces(s.x, s.q, s.box, p, with_abs=True)
    FP, TP = oracle.patchy_pair_scales(s.x, s.q, s.box, p)
    tol = 1 + 1e-13
    assert np.all(np.abs(F) <= FP * tol) and np.all(FP <= FA * tol)
    assert np.all(np.abs(T) <= TP * tol) and np.all(TP <= TA * tol)
    b = RATIO_BOUNDS[model]
    for term, pair in ((FA, FP), (TA, TP)):
        m = pair > 0
        ratio = term[m] / pair[m]
        assert np.median(ratio) <= b["median"]
        assert np.percentile(ratio, 99) <= b["p99"]
        assert term.sum() / pair.sum() <= b["total"]


# ---------------------------------------------------------------------------
# Generator margin
# ---------------------------------------------------------------------------

def _margin_numpy(x, L, radii):
    """min over pairs i < j with r < max(radii) + 1 and over the radii of
    |r - R|, from a full minimum-image distance matrix."""
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d * d).sum(-1))
    iu = np.triu_indices(len(x), 1)
    r = r[iu]
    r = r[r < max(radii) + 1.0]
    return min(np.abs(r - R).min() for R in radii)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pair_margin_brute_force(seed):
    """or_pair_margin (cell list) equals the numpy brute-force minimum on
    300-particle LJ and patchy states."""
    for name in ("lj_small", "patchy"):
        w = WORKLOADS[name].with_(n=300)
        s = make_state(w, seed)
        radii = [w.rcut, w.rcut + w.skin]
        got = oracle.pair_margin(s.x, s.box, radii)
        assert got == pytest.approx(_margin_numpy(s.x, s.box, radii), rel=1e-12, abs=1e-15)


def test_pair_margin_of_a_planted_pair():
    """A pair planted at r_c + 3e-10 (across the periodic boundary) in a
    dilute lattice gives a margin of 3e-10 to rounding: the margin sees both
    radii and the periodic image."""
    L, rc, rv = 20.0, 2.5, 2.8
    g = np.arange(4) * 5.0 + 1.0
    x = np.array([[a, b, c] for a in g for b in g for c in g])  # spacing 5 > rv + 1
    x[0] = [0.1, 1.0, 1.0]
    x[1] = [20.0 + 0.1 - rc - 3e-10, 1.0, 1.0]  # distance rc + 3e-10 through x = 0
    m = oracle.pair_margin(x, L, [rc, rv])
    assert m == pytest.approx(3e-10, rel=1e-4)
    assert m == pytest.approx(_margin_numpy(x, L, [rc, rv]), rel=1e-9)
