"""Cell orders of the locality study (host side, no GPU): every order is a
permutation of the cells; Morton is bit interleaving; the Hilbert curve visits
face neighbours one after the other and is not Morton."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def md():
    from paper_1401_4350_amd import md as m
    return m


def coords(nc, ranks):
    """Cell coordinates (x, y, z) in visiting order."""
    order = np.argsort(ranks)
    z, rem = np.divmod(order, nc * nc)
    y, x = np.divmod(rem, nc)
    return np.stack([x, y, z], 1)


@pytest.mark.parametrize("order", ["row_major", "row_major_gather", "morton", "hilbert"])
@pytest.mark.parametrize("nc", [1, 2, 3, 5, 8, 24])
def test_permutation(md, order, nc):
    r = md.cell_order_ranks(nc, order)
    assert np.array_equal(np.sort(r), np.arange(nc ** 3))


def test_row_major_identity(md):
    assert np.array_equal(md.cell_order_ranks(6, "row_major"), np.arange(216))


def test_morton_interleaves_bits(md):
    nc = 8
    r = md.cell_order_ranks(nc, "morton")
    for x, y, z in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (3, 5, 6), (7, 7, 7)]:
        want = sum(((x >> k) & 1) << (3 * k) | ((y >> k) & 1) << (3 * k + 1) |
                   ((z >> k) & 1) << (3 * k + 2) for k in range(3))
        assert r[(z * nc + y) * nc + x] == want


@pytest.mark.parametrize("nc", [2, 4, 8, 16])
def test_hilbert_steps_to_face_neighbours(md, nc):
    c = coords(nc, md.cell_order_ranks(nc, "hilbert"))
    assert np.array_equal(c[0], [0, 0, 0])
    steps = np.abs(np.diff(c, axis=0)).sum(1)
    assert np.all(steps == 1)  # a Hilbert curve moves one cell along one axis per step
    m = coords(nc, md.cell_order_ranks(nc, "morton"))
    if nc > 2:
        assert not np.all(np.abs(np.diff(m, axis=0)).sum(1) == 1)  # Morton jumps


@pytest.mark.parametrize("nc", [6, 24])
def test_hilbert_non_power_of_two_mostly_local(md, nc):
    """Ranked over the enclosing power-of-two cube, consecutive cells are
    still mostly face neighbours."""
    c = coords(nc, md.cell_order_ranks(nc, "hilbert"))
    steps = np.abs(np.diff(c, axis=0)).sum(1)
    assert np.mean(steps == 1) > 0.8


def test_invalid(md):
    with pytest.raises(md.MDError):
        md.cell_order_ranks(0, "hilbert")
    import ctypes
    out = np.zeros(8, np.int32)
    assert md.lib().md_cell_order_ranks(2, 9, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == -1
