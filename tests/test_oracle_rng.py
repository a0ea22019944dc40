"""Pins of the oracle's random draws (Sec. 2.3 distributions) against an
independent library generator and against the distributions' statistics."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox, sketch


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 123456789)])
def test_philox_matches_numpy_bitgenerator(key):
    # numpy's Philox (4x64, 10 rounds) increments its counter before each
    # block, so its b-th block is ours with counter b+1.
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.zeros(4, dtype=np.uint64))
    ref = g.random_raw(4 * 50)
    b = np.arange(1, 51, dtype=np.uint64)
    z = np.zeros_like(b)
    out = philox.philox4x64_10((b, z, z, z), (np.uint64(key[0]), np.uint64(key[1])))
    mine = np.stack(out, axis=1).reshape(-1)
    assert np.array_equal(mine, ref)


def test_philox_counter_words_layout():
    w = philox.words(9, 3, 10)
    out = philox.philox4x64_10((np.uint64(2), np.uint64(0), np.uint64(0), np.uint64(0)),
                               (np.uint64(9), np.uint64(3)))
    assert [int(x) for x in w[8:10]] == [int(out[0]), int(out[1])]


def test_mulhilo_exact():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2**63, size=200, dtype=np.uint64)
    hi, lo = philox.mulhilo(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2**64 - 1)


def test_signs_bit_layout_and_balance():
    N = 1 << 16
    d = sketch.srht_signs(11, N)
    w = philox.words(11, philox.STREAM_SIGNS, N // 64)
    for i in (0, 1, 63, 64, 1000, N - 1):
        bit = (int(w[i // 64]) >> (i % 64)) & 1
        assert d[i] == (-1.0 if bit else 1.0)
    assert set(np.unique(d)) == {-1.0, 1.0}
    # Rademacher: mean 0 with std 1/sqrt(N)
    assert abs(d.mean()) < 5 / np.sqrt(N)


def test_rows_are_a_uniform_sample_without_replacement():
    N, l = 64, 8
    counts = np.zeros(N)
    for seed in range(2000):
        r = sketch.srht_rows(seed, N, l)
        assert len(np.unique(r)) == l and np.all(np.diff(r) > 0)
        assert r.min() >= 0 and r.max() < N
        counts[r] += 1
    # chi-square test of uniform inclusion frequency l/N
    expected = 2000 * l / N
    chi2 = np.sum((counts - expected) ** 2 / expected)
    assert stats.chi2.sf(chi2, N - 1) > 1e-4


def test_rows_are_smallest_keys():
    N, l = 1000, 17
    keys = philox.words(4, philox.STREAM_ROWKEYS, N)
    r = sketch.srht_rows(4, N, l)
    thresh = np.sort(keys)[l - 1]
    assert np.all(keys[r] <= thresh)
    assert np.sum(keys <= thresh) == l


def test_gaussian_moments_and_normality():
    l, nt = 40, 5000
    Om = sketch.gaussian_omega(3, l, nt)
    assert Om.shape == (l, nt)
    g = Om.reshape(-1) * np.sqrt(l)
    assert abs(g.mean()) < 5 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * np.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-4


def test_gaussian_column_major_entry_order():
    l, nt = 3, 4
    Om = sketch.gaussian_omega(8, l, nt)
    w = philox.words(8, philox.STREAM_GAUSS, 2 * l * nt)
    k, i = 2, 1
    e = k + l * i
    a, b = int(w[2 * e]), int(w[2 * e + 1])
    u1 = ((a >> 11) + 1) * 2.0 ** -53
    u2 = (b >> 11) * 2.0 ** -53
    g = np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)
    assert Om[k, i] == g / np.sqrt(l)
