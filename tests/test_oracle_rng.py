"""Pins of the oracle's counter-based generator and the conversions built on it.

NumPy's Philox bit generator is an independent implementation of the same
Philox4x64-10 definition; it advances its 256-bit counter by one before
producing each block, so block(c) there equals philox4x64_10(c + 1).
"""
import math

import numpy as np
import pytest

from oracle import philox
from oracle.lattice import Lattice, init_tensors, neel, neel_shuffled


def _numpy_block(counter, key):
    c = sum(int(v) << (64 * i) for i, v in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & philox.MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return tuple(int(v) for v in bg.random_raw(4))


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 2, 3, 4), (5, 6)),
    ((2**64 - 1, 7, 2**63, 12345), (2**64 - 1, 2**64 - 1)),
    ((4095, 19, 111, philox.TAG_METRO), (1908, 3)),
    ((0, 0, 0, 0), (0xDEADBEEF, 0)),
])
def test_philox_matches_numpy(counter, key):
    assert philox.philox4x64_10(counter, key) == _numpy_block(counter, key)


def test_philox_random_counters_match_numpy():
    rng = np.random.default_rng(7)
    for _ in range(50):
        counter = tuple(int(v) for v in rng.integers(0, 2**63, size=4))
        key = tuple(int(v) for v in rng.integers(0, 2**63, size=2))
        assert philox.philox4x64_10(counter, key) == _numpy_block(counter, key)


def test_uniform53_exact_range():
    assert philox.uniform53(0) == 0.0
    assert philox.uniform53(philox.MASK64) == 1.0 - 2.0 ** -53
    assert philox.uniform53(1 << 11) == 2.0 ** -53


def test_bounded_index_is_floor():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        w = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        n = int(rng.integers(1, 2048))
        u = philox.uniform53(w)
        # u*n is exact in binary64 when n < 2^11 and u has 53 significant bits only if
        # the product fits; compare against exact rational floor instead.
        exact = ((w >> 11) * n) // (1 << 53)
        assert philox.bounded_index(w, n) == exact
        assert exact == math.floor(u * n) or abs(u * n - round(u * n)) < 1e-12


def test_gaussian_moments():
    key = (11, 0)
    z = np.array([philox.gaussian((i, 0, 0, philox.TAG_INIT), key) for i in range(20000)])
    assert abs(z.mean()) < 0.03
    assert abs(z.var() - 1.0) < 0.04
    assert abs(np.mean(z ** 4) - 3.0) < 0.2


def test_init_tensor_scale_and_determinism():
    lat = Lattice(3, 3, 2, 4)
    a = init_tensors(lat, seed=5)
    b = init_tensors(lat, seed=5)
    c = init_tensors(lat, seed=6)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert len(a) == lat.Np
    # scale 1/D^2 on unit normals
    assert abs(np.std(a) * lat.D ** 2 - 1.0) < 0.2
    p = init_tensors(lat, seed=5, perturb=1e-2)
    assert 0 < np.max(np.abs(p - a)) < 0.1


def test_neel_and_shuffle():
    lat = Lattice(4, 6, 2, 4)
    s = neel(lat).reshape(4, 6)
    assert s[0, 0] == 0 and s[0, 1] == 1 and s[1, 0] == 1
    seen = set()
    for chain in range(20):
        sh = neel_shuffled(lat, 9359, 0, chain)
        assert sh.sum() == lat.N // 2
        seen.add(sh.tobytes())
        assert np.array_equal(sh, neel_shuffled(lat, 9359, 0, chain))
    assert len(seen) == 20


def _arrangement_counts(lat, n_chains, seed=9359):
    counts = {}
    for chain in range(n_chains):
        k = neel_shuffled(lat, seed, 0, chain).tobytes()
        counts[k] = counts.get(k, 0) + 1
    return counts


def _chi2_uniform_pvalue(counts, n_cells, n):
    from scipy import stats
    obs = np.zeros(n_cells)
    obs[:len(counts)] = list(counts.values())
    return stats.chisquare(obs, np.full(n_cells, n / n_cells)).pvalue


def test_neel_shuffle_is_uniform_over_the_sector():
    """A uniform permutation of the Neel list gives every S^z = 0 arrangement with
    probability 1 / C(N, N/2).  On a 2x3 lattice (20 arrangements) the shuffled
    starts of 6000 chains pass a chi-square test of uniformity, while the same
    shuffle with a planted Sattolo index range (j < i, which draws only N-cycles
    and can never return the Neel arrangement itself) fails it."""
    from math import comb
    lat = Lattice(2, 3, 2, 4)
    n, cells = 6000, comb(6, 3)
    counts = _arrangement_counts(lat, n)
    assert len(counts) == cells
    assert _chi2_uniform_pvalue(counts, cells, n) > 1e-3
    exact = philox.bounded_index
    philox.bounded_index = lambda word, m: exact(word, m - 1)  # j in [0, i): Sattolo's algorithm
    try:
        planted = _arrangement_counts(lat, n)
    finally:
        philox.bounded_index = exact
    assert neel(lat).tobytes() not in planted
    assert _chi2_uniform_pvalue(planted, cells, n) < 1e-6
