"""Seeded generator: determinism and the stated recipe (no GPU)."""
import math

import numpy as np

from paper_1401_4350_amd.inputs import WORKLOADS, lattice, make_state


def test_seed_determinism_and_attempts():
    w = WORKLOADS["lj_small"].with_(n=1000)
    a, b = make_state(w, 7), make_state(w, 7)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    c = make_state(w, 7, attempt=1)
    assert not np.array_equal(a.x, c.x)


def test_density_temperature_momentum():
    for name in ("lj_small", "patchy"):
        w = WORKLOADS[name].with_(n=3000)
        s = make_state(w, 1)
        assert s.box == (w.n / w.rho) ** (1 / 3)
        assert np.all(s.x >= 0) and np.all(s.x < s.box)
        assert np.abs(s.v.sum(0)).max() < 1e-9
        t = w.mass * (s.v ** 2).sum() / (3 * w.n - 3)
        assert abs(t - w.temp) < 1e-12
        if w.pot == "patchy":
            assert np.allclose(np.linalg.norm(s.q, axis=1), 1.0)
            assert s.angmom.shape == (w.n, 3)


def test_lattice_partial_fill():
    """Non-cube N fills the first N sites of a ceil(N^(1/3))^3 lattice."""
    x = lattice(131072, 64.0)
    m = 51
    assert math.ceil(131072 ** (1 / 3)) == m
    a = 64.0 / m
    assert np.allclose(x[:3, 0], [0.5 * a, 1.5 * a, 2.5 * a])
    assert x[:, 2].max() < 64.0
    assert len(np.unique(np.round(x / a - 0.5).astype(int), axis=0)) == 131072
    # perfect cubes use the exact side
    assert np.isclose(lattice(4096, 16.0)[:, 0].max(), 15.5)


def test_chain_columns_geometry():
    """The two-patch workload's sites: columns along z spaced box / floor(box /
    1.04) >= 1.04, on a square (x, y) grid, all inside the box, no two sites
    closer than the column spacing."""
    import math
    from paper_1401_4350_amd.inputs import chain_columns
    for n, box in ((2000, 15.874), (1001, 12.6), (250, 7.94)):
        x = chain_columns(n, box)
        assert x.shape == (n, 3)
        assert (x >= 0).all() and (x < box).all()
        nz = int(box // 1.04)
        b = box / nz
        assert b >= 1.04
        # along a column, consecutive sites are b apart
        col = x[:nz]
        assert np.allclose(np.diff(col[:, 2]), b)
        assert np.allclose(col[:, :2], col[0, :2])
        # the columns' (x, y) spacing is no smaller than b for these densities
        xy = np.unique(np.round(x[:, :2], 9), axis=0)
        d = np.abs(xy[:, None, :] - xy[None, :, :]).max(axis=2)
        d[np.diag_indices_from(d)] = math.inf
        assert d.min() >= b - 1e-9


def test_patchy_paper_orientations():
    """About 70 % of the two-patch particles start with the body z axis within
    a small tilt of the lab z axis (the chain direction), the rest uniform."""
    from paper_1401_4350_amd.inputs import WORKLOADS, make_state
    w = WORKLOADS["patchy_paper"].with_(n=20000)
    s = make_state(w, 3)
    q = s.q
    # body z axis in the lab frame: third column of R(q)
    zz = 1 - 2 * (q[:, 1] ** 2 + q[:, 2] ** 2)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0)
    frac = np.mean(zz > np.cos(0.6))
    assert 0.68 < frac < 0.76
