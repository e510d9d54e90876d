"""Pins of the oracle's counter-based random numbers.

The Philox4x64-10 block function is checked against numpy's independent
implementation of the same generator (numpy.random.Philox), word for word;
the normals against the standard normal distribution (moments, KS).
"""
import numpy as np
import pytest
from scipy import stats


def _numpy_block(ctr, key):
    # numpy increments the 256-bit counter before producing each block
    c = np.array(ctr, dtype=object)
    val = sum(int(c[i]) << (64 * i) for i in range(4)) - 1
    val %= 1 << 256
    words = np.array([(val >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.asarray(key, dtype=np.uint64), counter=words)
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [5, 7]),
    ([17, 3, 999, 0x203], [3001, 0]),
    ([2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1], [2**64 - 1, 2**64 - 1]),
    ([123456789, 42, 2**40 + 5, 0x0E04], [0xDEADBEEF, 0x12345]),
])
def test_philox_matches_numpy(orc, ctr, key):
    got = orc.philox4x64_10(ctr, key)
    ref = _numpy_block(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_many_counters_match_numpy(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert np.array_equal(orc.philox4x64_10(ctr, key), _numpy_block(ctr, key))


def test_u01_open_interval_and_resolution(orc):
    assert orc.u01(0) == 0.5 * 2.0**-53
    assert 0.0 < orc.u01(0) < 1.0
    assert orc.u01(2**64 - 1) <= 1.0
    # 53 leading bits: words differing only in the low 11 bits give the same uniform
    assert orc.u01(0xABCDEF0123456000) == orc.u01(0xABCDEF01234567FF)


def test_normals_distribution(orc):
    z = np.concatenate([orc.normals(3001, m, 7, 1, 0, 1000) for m in range(200)])
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # fourth moment of a standard normal is 3
    assert abs((z**4).mean() - 3.0) < 0.1


def test_normals_streams_are_distinct_and_reproducible(orc):
    a = orc.normals(1, 0, 0, 1, 0, 64)
    b = orc.normals(1, 0, 0, 2, 0, 64)
    c = orc.normals(1, 0, 0, 1, 1, 64)
    d = orc.normals(1, 1, 0, 1, 0, 64)
    e = orc.normals(1, 0, 1, 1, 0, 64)
    for other in (b, c, d, e):
        assert not np.allclose(a, other)
    assert np.array_equal(a, orc.normals(1, 0, 0, 1, 0, 64))
    # a prefix of a longer request is the shorter request (blocks are per 8 dims)
    assert np.array_equal(orc.normals(1, 0, 0, 1, 0, 10), a[:10])


def test_normals_block_layout(orc):
    # block j of the stream fills dims 8j..8j+7; word k gives (U_a, U_b) from its
    # high and low halves, (w + 1/2) / 2^32, and Box-Muller makes the pair
    w = orc.philox4x64_10([5, 1, 9, 1 | (3 << 8)], [77, 0])
    ref = []
    for v in w:
        ua = ((int(v) >> 32) + 0.5) / 2.0**32
        ub = ((int(v) & 0xFFFFFFFF) + 0.5) / 2.0**32
        r = np.sqrt(-2 * np.log(ua))
        ref += [r * np.cos(2 * np.pi * ub), r * np.sin(2 * np.pi * ub)]
    z = orc.normals(77, 5, 9, 1, 3, 20)
    np.testing.assert_allclose(z[8:16], ref, rtol=1e-15, atol=1e-15)


def test_mh_uniform_stream(orc):
    w = orc.philox4x64_10([3, 0, 11, 4], [9, 0])
    assert orc.mh_uniform(9, 3, 11) == orc.u01(int(w[0]))
    us = np.array([orc.mh_uniform(9, m, 11) for m in range(5000)])
    assert stats.kstest(us, "uniform").pvalue > 1e-3
