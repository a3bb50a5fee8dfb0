"""Pins of the oracle's generator variants.

Tyche-i: its round (MIX-i) inverts Tyche's MIX, which is itself pinned to
OpenSSL's ChaCha20 quarter round; twenty pinned MIX rounds take a Tyche-i
state back to the raw seeding words (whose constants are checked against
their closed forms here, in exact arithmetic); after j outputs, 20 + j MIX
rounds do the same, so a Tyche-i stream is Tyche's state orbit walked
backwards; the stream layout is Tyche's tile layout.
Squares64: the high half of every output is the separately transcribed
Squares32 output of the same counter and key (the two share rounds 1-4);
the stream interleaves the halves of consecutive calls; avalanche and byte
frequencies.  Which Tyche-i word is output, and Squares64's low half, are
parity unpinned (no implementation in the container)."""
import ctypes as C
import math
import random
from fractions import Fraction

import numpy as np
import pytest

M32 = 0xFFFFFFFF


def _floor_2p32_over_phi():
    # 2^32 / phi = 2^31 (sqrt 5 - 1): floor by integer square root
    return (math.isqrt(5 * 2**62) - 2**31)


def _floor_2p32_over_pi():
    # pi bracketed by Machin's series to 60 digits in exact rationals
    def atan_inv(n, terms=60):
        s, x = Fraction(0), Fraction(1, n)
        for k in range(terms):
            s += (-1) ** k * x ** (2 * k + 1) / (2 * k + 1)
        return s
    pi = 16 * atan_inv(5) - 4 * atan_inv(239)
    return math.floor(Fraction(2**32) / pi)


def test_closed_form_constants():
    assert _floor_2p32_over_phi() == 2654435769
    assert _floor_2p32_over_pi() == 1367130551


def test_mix_i_inverts_mix(O):
    r = random.Random(71)
    for _ in range(2000):
        s = [r.getrandbits(32) for _ in range(4)]
        assert O.tyche_mix_i(O.tyche_mix(s)) == s
        assert O.tyche_mix(O.tyche_mix_i(s)) == s
    # and it is not MIX itself
    s = [1, 2, 3, 4]
    assert O.tyche_mix_i(s) != O.tyche_mix(s)


def test_tyche_i_orbit_runs_back_to_the_seeding_words(O):
    """After seeding and j outputs, 20 + j rounds of the pinned MIX return the
    raw state (seed hi, seed lo, C0 ^ substream, D0 ^ counter)."""
    L = O.lib()
    r = random.Random(72)
    for _ in range(30):
        seed, cx, dx = r.getrandbits(64), r.getrandbits(32), r.getrandbits(32)
        raw = [seed >> 32, seed & M32, _floor_2p32_over_phi() ^ cx, _floor_2p32_over_pi() ^ dx]
        st = (C.c_uint32 * 4)()
        L.oracle_tyche_i_init(seed, cx, dx, st)
        for j in range(6):
            s = list(st)
            for _ in range(20 + j):
                s = O.tyche_mix(s)
            assert s == raw, j
            w = L.oracle_tyche_i_next(st)
            assert w == st[1]


def test_tyche_i_layout_is_tyche_tile_layout(O):
    seed, ctr = 0x0DDBA11, 5
    words = O.fill(O.TYCHE_I, O.U32, seed, ctr, 0, 2 * 16384)
    for t, l in [(0, 0), (0, 63), (1, 17)]:
        sub = O.tyche_i_stream(seed, t * 64 + l, ctr, 256)
        for k in (0, 1, 63):
            for w in range(4):
                assert words[t * 16384 + (k * 64 + l) * 4 + w] == sub[4 * k + w], (t, l, k, w)
    # substream 0 is the textbook instance; the stream differs from Tyche's
    assert list(words[:4]) == O.tyche_i_stream(seed, 0, ctr, 4)
    assert not np.array_equal(words[:64], O.fill(O.TYCHE, O.U32, seed, ctr, 0, 64))


def test_squares64_high_half_is_squares32(O):
    r = random.Random(73)
    for _ in range(3000):
        ctr, key = r.getrandbits(64), r.getrandbits(64) | 1
        assert O.squares64(ctr, key) >> 32 == O.squares32(ctr, key)


def test_squares64_layout(O):
    seed, ctr, off, n = 0xFACE, 9, 1001, 5000
    key = O.squares_key(seed)
    got = O.fill(O.SQUARES64, O.U32, seed, ctr, off, n)
    for j in list(range(0, n, 71)) + [n - 1]:
        p = off + j
        v = O.squares64((ctr << 32) | (p // 2), key)
        assert got[j] == ((v >> 32) if p & 1 else (v & M32)), j
    last = O.fill(O.SQUARES64, O.U32, seed, ctr, 2**32 - 2, 2)
    v = O.squares64((ctr << 32) | (2**31 - 1), key)
    assert list(last) == [v & M32, v >> 32]


def test_squares64_avalanche(O):
    r = random.Random(74)
    key = O.squares_key(12345)
    flips = []
    for _ in range(400):
        c = r.getrandbits(63)
        b = r.randrange(63)
        flips.append(bin(O.squares64(c, key) ^ O.squares64(c ^ (1 << b), key)).count("1"))
    m = sum(flips) / len(flips)
    assert abs(m - 32) < 5 * 4 / math.sqrt(len(flips))


@pytest.mark.parametrize("gen", [7, 8])
def test_variant_streams_statistics(O, gen):
    from scipy import stats
    w = O.fill(gen, O.U32, 2023, 3, 0, 1 << 20)
    assert stats.chisquare(np.bincount(w.view(np.uint8), minlength=256))[1] > 1e-4
    u = (w >> 8) / 2**24
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5 / math.sqrt(u.size)
    # different counters give unrelated streams
    v = O.fill(gen, O.U32, 2023, 4, 0, 1 << 16)
    assert abs(np.corrcoef(w[:1 << 16] >> 8, v >> 8)[0, 1]) < 5 / math.sqrt(1 << 16)


def test_variants_through_every_oracle_entry_point(O):
    for gen in (7, 8, 9):
        f = O.fill(gen, O.F32_UNIFORM, 1, 2, 3, 1000)
        at = O.samples_at(gen, O.F32_UNIFORM, 1, np.full(3, 2, np.uint32),
                          np.array([3, 500, 1002], np.uint64))
        assert np.array_equal(at, f[[0, 497, 999]])
        m = O.fill_multi(gen, O.U32, 1, 2, 3, 5, 40).reshape(3, 40)
        assert np.array_equal(m[2], O.fill(gen, O.U32, 1, 4, 5, 40))
        ps = O.particle_streams(gen, 10, 4, 3, 6, 2).reshape(2, 4, 3)
        assert np.array_equal(ps[1, 2], O.fill(gen, O.U32, 12, 7, 0, 3))
    with pytest.raises(ValueError):
        O.fill(10, O.U32, 1, 2, 3, 10)
