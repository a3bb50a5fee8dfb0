"""Pins of the oracle's Philox2x32-10 (the two-word Philox of Salmon et al.,
SC'11) and of its stream layout.  No implementation of Philox2x32 is at hand
in this environment, so its constants are parity unpinned; what is pinned:
ten inverse rounds, written here from the round's definition, take every
output back to its counter (the rounds form a bijection of the stated shape),
2^20 enumerated counters give 2^20 distinct blocks, the stream layout, the
32-bit seed limit, and avalanche and byte statistics."""
import math
import random

import numpy as np
import pytest

M = 0xD256D193
W = 0x9E3779B9
MASK = 0xFFFFFFFF
MINV = pow(M, -1, 1 << 32)


def _invert(out, key):
    """Undo ten rounds: the second word is the low half of M * a, so
    a = lo * M^-1 (M is odd); the first word is hi(M * a) ^ b ^ k, so b
    follows once a is known.  Keys are taken in reverse order."""
    a, b = out
    for r in reversed(range(10)):
        k = (key + r * W) & MASK
        prev_a = (b * MINV) & MASK
        hi = (M * prev_a) >> 32
        prev_b = a ^ hi ^ k
        a, b = prev_a, prev_b
    return [a, b]


def test_inverse_rounds_recover_the_counter(O):
    r = random.Random(91)
    cases = [([0, 0], 0), ([MASK, MASK], MASK), ([1, 0], 0), ([0, 1], 0)]
    cases += [([r.getrandbits(32), r.getrandbits(32)], r.getrandbits(32)) for _ in range(2000)]
    for ctr, key in cases:
        out = O.philox2x32_10(ctr, key)
        assert _invert(out, key) == ctr, (ctr, key)
    # a different key does not invert the same output back
    out = O.philox2x32_10([5, 6], 7)
    assert _invert(out, 8) != [5, 6]


def test_enumerated_counters_give_distinct_blocks(O):
    w = O.fill(O.PHILOX2X32, O.U32, 0xC0FFEE, 3, 0, 1 << 21)  # blocks 0 .. 2^20 - 1
    pairs = w.view(np.uint64)
    assert np.unique(pairs).size == 1 << 20


def test_stream_layout(O):
    r = random.Random(92)
    for _ in range(20):
        seed, ctr = r.getrandbits(32), r.getrandbits(32)
        off = r.randrange(0, 2**32 - 5000)
        got = O.fill(O.PHILOX2X32, O.U32, seed, ctr, off, 4099)
        for j in list(range(0, 4099, 97)) + [4098]:
            p = off + j
            assert got[j] == O.philox2x32_10([p // 2, ctr], seed)[p % 2], (seed, ctr, p)
    # the last two words of the stream: block 2^31 - 1
    last = O.fill(O.PHILOX2X32, O.U32, 77, 5, 2**32 - 2, 2)
    assert list(last) == O.philox2x32_10([2**31 - 1, 5], 77)


def test_seed_limit(O):
    O.fill(O.PHILOX2X32, O.U32, MASK, 1, 0, 8)
    with pytest.raises(ValueError):
        O.fill(O.PHILOX2X32, O.U32, 1 << 32, 1, 0, 8)
    with pytest.raises(ValueError):
        O.fill_multi(O.PHILOX2X32, O.U32, 1 << 32, 1, 2, 0, 8)
    with pytest.raises(ValueError):
        O.fill_range(O.PHILOX2X32, 1 << 32, 1, 1, 0, 8, 0, 10)
    O.particle_streams(O.PHILOX2X32, MASK - 3, 4, 3, 0, 2)
    with pytest.raises(ValueError):
        O.particle_streams(O.PHILOX2X32, MASK - 3, 5, 3, 0, 2)
    # other generators keep taking 64-bit seeds
    O.fill(O.PHILOX, O.U32, 1 << 40, 1, 0, 8)


def test_avalanche(O):
    r = random.Random(93)
    flips = []
    for _ in range(600):
        c = [r.getrandbits(32), r.getrandbits(32)]
        k = r.getrandbits(32)
        base = O.philox2x32_10(c, k)
        which = r.randrange(3)
        bit = 1 << r.randrange(32)
        if which == 2:
            other = O.philox2x32_10(c, k ^ bit)
        else:
            c2 = list(c)
            c2[which] ^= bit
            other = O.philox2x32_10(c2, k)
        flips.append(bin(base[0] ^ other[0]).count("1") + bin(base[1] ^ other[1]).count("1"))
    m = sum(flips) / len(flips)
    assert abs(m - 32) < 5 * 4 / math.sqrt(len(flips))


def test_stream_statistics(O):
    from scipy import stats
    w = O.fill(O.PHILOX2X32, O.U32, 2023, 3, 0, 1 << 20)
    assert stats.chisquare(np.bincount(w.view(np.uint8), minlength=256))[1] > 1e-4
    u = (w >> 8) / 2**24
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5 / math.sqrt(u.size)
    v = O.fill(O.PHILOX2X32, O.U32, 2023, 4, 0, 1 << 16)
    assert abs(np.corrcoef(w[:1 << 16] >> 8, v >> 8)[0, 1]) < 5 / math.sqrt(1 << 16)
