"""Pins of the oracle's integer samples in [lo, hi) (a reading of section 3's
standard-distribution use): power-of-two ranges reduce to the top bits of the
high word; the preimage thresholds ceil(v 2^64 / r) of every value, computed
in exact integer arithmetic, land where they must; a range where the
remainder method would be off by 2:1 has the exact frequencies; the stream
layout agrees with the pinned word stream (words 2p and 2p+1 for sample p)."""
import math

import numpy as np
import pytest

I32_MIN, I32_MAX = -2**31, 2**31 - 1


def test_power_of_two_ranges(O):
    """r = 2^k: floor(x 2^k / 2^64) is the top k bits of x, i.e. of w1."""
    rng = np.random.default_rng(1)
    for k in range(32):
        for lo in (0, -7, I32_MIN, I32_MAX - 2**k):
            if lo + 2**k > I32_MAX:
                continue  # hi must be an int32
            for _ in range(20):
                w0, w1 = (int(v) for v in rng.integers(0, 2**32, 2))
                assert O.range_i32(w0, w1, lo, lo + 2**k) == lo + (w1 >> (32 - k)), (k, lo)


def test_preimage_thresholds(O):
    """The smallest x giving value v is ceil(v 2^64 / r): x there gives v and
    x - 1 gives v - 1.  Checks the scaling, the word order and the offset in
    one go; it also shows the preimages of neighbouring values differ in
    size by at most one (the bias bound)."""
    rng = np.random.default_rng(2)
    rs = [1, 2, 3, 5, 6, 7, 1000, 2**31 - 1, 2**31 + 1, 3 * 2**30, 2**32 - 1]
    rs += [int(v) for v in rng.integers(1, 2**32, 40)]
    for r in rs:
        lo = I32_MIN if r > 2**31 else int(rng.integers(I32_MIN, I32_MAX - r + 2))
        hi = lo + r
        for v in {0, 1, r - 1, r // 2, int(rng.integers(0, r))}:
            if v >= r:
                continue
            x = -((-v * 2**64) // r)  # ceil
            assert O.range_i32(x & 0xFFFFFFFF, x >> 32, lo, hi) == lo + v, (r, v)
            if v > 0:
                y = x - 1
                assert O.range_i32(y & 0xFFFFFFFF, y >> 32, lo, hi) == lo + v - 1, (r, v)
            nxt = -((-(v + 1) * 2**64) // r)
            assert abs((nxt - x) - 2**64 // r) <= 1
        assert O.range_i32(0, 0, lo, hi) == lo
        assert O.range_i32(0xFFFFFFFF, 0xFFFFFFFF, lo, hi) == hi - 1


def test_full_int32_span(O):
    got = O.fill_range(0, 3, 4, 1, 0, 1 << 16, I32_MIN, I32_MAX)
    assert got.min() >= I32_MIN and got.max() < I32_MAX
    assert got.min() < -2**31 + 2**20 and got.max() > 2**31 - 2**20


@pytest.mark.parametrize("gen", range(10))
def test_no_remainder_bias(O, gen):
    """r = 3 * 2^30: the remainder of one 32-bit word would put half of all
    samples in the lowest third; here each third holds a third."""
    n = 1 << 20
    lo = I32_MIN
    got = O.fill_range(gen, 0xC0FFEE, 9, 1, 0, n, lo, lo + 3 * 2**30).astype(np.int64) - lo
    frac = np.bincount(got >> 30, minlength=3) / n
    sd = math.sqrt(2 / 9 / n)
    assert np.all(np.abs(frac - 1 / 3) < 5 * sd), frac


@pytest.mark.parametrize("gen", range(10))
def test_die_frequencies(O, gen):
    from scipy import stats
    got = O.fill_range(gen, 77, 0, 1, 1000, 600000, 1, 7)
    assert got.min() == 1 and got.max() == 6
    assert stats.chisquare(np.bincount(got, minlength=7)[1:])[1] > 1e-4


@pytest.mark.parametrize("gen", range(10))
def test_layout_follows_the_word_stream(O, gen):
    """Sample p of a stream is built from words 2p and 2p+1 of the same
    stream; many streams are counters ctr0 + i."""
    seed, ctr, off, n = 0x1234_5678_9ABC, 17, 4093, 9000
    if gen == O.PHILOX2X32:
        seed &= 0xFFFFFFFF  # a 32-bit key
    w = O.fill(gen, O.U32, seed, ctr, 2 * off, 2 * n)
    ref = [O.range_i32(w[2 * j], w[2 * j + 1], -1000, 999) for j in range(0, n, 97)]
    got = O.fill_range(gen, seed, ctr, 1, off, n, -1000, 999)
    assert list(got[::97]) == ref
    multi = O.fill_range(gen, seed, ctr, 5, 3, 301, -1000, 999).reshape(5, 301)
    for i in range(5):
        assert np.array_equal(multi[i], O.fill_range(gen, seed, ctr + i, 1, 3, 301, -1000, 999))
    # the last samples of the stream
    last = O.fill_range(gen, seed, ctr, 1, 2**31 - 3, 3, 0, 2**31 - 1)
    w = O.fill(gen, O.U32, seed, ctr, 2**32 - 6, 6)
    assert list(last) == [O.range_i32(w[2 * j], w[2 * j + 1], 0, 2**31 - 1) for j in range(3)]


def test_range_errors(O):
    O.fill_range(0, 0, 0, 1, 2**31, 0, 0, 1)
    O.fill_range(0, 0, 2**32 - 2, 2, 0, 4, 0, 1)
    for args in [(0, 0, 0, 1, 0, 4, 5, 5), (0, 0, 0, 1, 0, 4, 6, 5), (10, 0, 0, 1, 0, 4, 0, 1),
                 (0, 0, 0, 1, 2**31 - 3, 4, 0, 1), (0, 0, 2**32 - 2, 3, 0, 4, 0, 1)]:
        with pytest.raises(ValueError):
            O.fill_range(*args)
