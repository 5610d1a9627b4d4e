"""Pins of the oracle's stochastic thermostat (Methods section: NVT runs with
the Brownian thermostat it cites, in the reading that each particle's momenta
are redrawn from the Maxwell-Boltzmann distribution with a fixed probability).

The generator is pinned to numpy's own Philox4x64-10 bit generator (an
independent implementation of the same published definition); the thermostat
to what the distribution fixes: the refreshed fraction is binomial, the new
velocities and angular momenta are normal with variances T/m and I T, and
the particles not drawn keep their momenta bit for bit."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


def numpy_philox_block(ctr, key):
    """numpy's Philox advances its counter by one before each block."""
    c = [int(w) for w in ctr]
    # counter - 1 with borrow across the four words
    for k in range(4):
        if c[k] > 0:
            c[k] -= 1
            break
        c[k] = (1 << 64) - 1
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                          key=np.array([int(w) for w in key], dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [5, 7]),
    ([12345, 678, 1, 0], [0xDEADBEEF, 0]),
    ([0, 1, 0, 0], [2 ** 64 - 1, 2 ** 63]),
    ([2 ** 64 - 1, 2 ** 64 - 1, 3, 9], [42, 0]),
])
def test_philox_equals_numpy(ctr, key):
    got = oracle.philox4x64(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(got, numpy_philox_block(ctr, key))


def test_philox_stream_equals_numpy():
    bg = np.random.Philox(counter=[0, 0, 0, 0], key=[11, 3])
    raw = bg.random_raw(4 * 64).astype(np.uint64).reshape(64, 4)
    for c in range(64):
        assert np.array_equal(oracle.philox4x64([c + 1, 0, 0, 0], [11, 3]), raw[c])


def _momenta(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 3)), rng.normal(size=(n, 3))


def test_probability_zero_and_one():
    v, L = _momenta(1000, 1)
    v0, L0, hits = oracle.thermostat(v, L, 0.15, 0.0, seed=3, counter=0)
    assert hits == 0 and np.array_equal(v0, v) and np.array_equal(L0, L)
    v1, L1, hits = oracle.thermostat(v, L, 0.15, 1.0, seed=3, counter=0)
    assert hits == 1000
    assert not np.any(v1 == v) and not np.any(L1 == L)


def test_maxwell_boltzmann():
    n, T, m, I, p = 200000, 0.15, 2.0, 0.4, 0.3
    v, L = _momenta(n, 2)
    v2, L2, hits = oracle.thermostat(v, L, T, p, seed=9, counter=17, mass=m, inertia=I)
    sd = math.sqrt(n * p * (1 - p))
    assert abs(hits - n * p) < 5 * sd
    changed = np.any(v2 != v, axis=1)
    assert changed.sum() == hits
    # particles not drawn keep their momenta exactly
    assert np.array_equal(v2[~changed], v[~changed])
    assert np.array_equal(L2[~changed], L[~changed])
    assert np.all(L2[changed] != L[changed])
    for arr, var in ((v2[changed], T / m), (L2[changed], I * T)):
        x = arr.ravel() / math.sqrt(var)
        k = x.size
        assert abs(x.mean()) < 5 / math.sqrt(k)
        assert abs(x.var() - 1) < 5 * math.sqrt(2 / k)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    # components uncorrelated (the pairs of one Box-Muller draw included)
    c = np.corrcoef(np.hstack([v2[changed], L2[changed]]).T)
    assert np.abs(c - np.eye(6)).max() < 5 / math.sqrt(hits)


def test_deterministic_and_counter_dependent():
    v, L = _momenta(5000, 3)
    a = oracle.thermostat(v, L, 1.0, 0.5, seed=1, counter=4)
    b = oracle.thermostat(v, L, 1.0, 0.5, seed=1, counter=4)
    c = oracle.thermostat(v, L, 1.0, 0.5, seed=1, counter=5)
    d = oracle.thermostat(v, L, 1.0, 0.5, seed=2, counter=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    sel = [np.any(x[0] != v, axis=1) for x in (a, c, d)]
    # independent draws: about a quarter of the particles in both selections
    for s in sel[1:]:
        both = np.mean(sel[0] & s)
        assert abs(both - 0.25) < 5 * math.sqrt(0.25 * 0.75 / 5000)


def test_lj_without_angular_momenta():
    v, _ = _momenta(3000, 4)
    v2, L2, hits = oracle.thermostat(v, None, 1.5, 0.2, seed=5, counter=0)
    assert L2 is None and 0 < hits < 3000
    # the same draws as with angular momenta present
    v3, _, hits3 = oracle.thermostat(v, np.zeros((3000, 3)), 1.5, 0.2, seed=5, counter=0)
    assert hits3 == hits and np.array_equal(v2, v3)
