"""Pins of the oracle's float64 Box-Muller normals: its ln, cos and sin
against 60-digit decimal arithmetic (decimal's correctly rounded ln and
sqrt; pi from Machin's formula; cos and sin from their Taylor series at the
full angle, with no reduction), within stated ulp bounds, on edge arguments
and random ones over every binade; exact values at quarter turns and at
u1 = 1; the stream layout against the pinned words; moments, the
Kolmogorov-Smirnov distance and pair independence of many samples."""
import math
from decimal import Decimal, localcontext
from fractions import Fraction

import numpy as np
import pytest

PREC = 60


def _pi():
    """Machin: pi = 16 atan(1/5) - 4 atan(1/239), atan by its series."""
    def atan_inv(n):
        x = Decimal(1) / n
        x2, term, total, k = x * x, x, x, 1
        while True:
            term *= -x2
            k += 2
            add = term / k
            if abs(add) < Decimal(10) ** (-PREC - 5):
                return total
            total += add
    return 16 * atan_inv(5) - 4 * atan_inv(239)


def _cos_sin(theta):
    """Taylor series of cos and sin at theta (|theta| < 7), no reduction."""
    c, s, term, n = Decimal(0), Decimal(0), Decimal(1), 0
    while True:
        if n % 4 == 0:
            c += term
        elif n % 4 == 1:
            s += term
        elif n % 4 == 2:
            c -= term
        else:
            s -= term
        n += 1
        term = term * theta / n
        if n > 10 and abs(term) < Decimal(10) ** (-PREC - 5):
            return c, s


def _ulp(v):
    v = abs(float(v))
    return 2.0 ** (math.frexp(v)[1] - 53) if v else 2.0 ** -1074


def _err_ulps(got, exact):
    return abs(Fraction(got) - Fraction(exact)) / Fraction(_ulp(exact))


@pytest.fixture(scope="module")
def PI():
    with localcontext() as ctx:
        ctx.prec = PREC
        return _pi()


def test_pi_is_pi(PI):
    assert float(PI) == math.pi
    assert str(PI).startswith("3.14159265358979323846264338327950288419716939937510")


def test_ln_u1_edges(O):
    assert O.ln_u1_f64(2**53) == 0.0 and math.copysign(1, O.ln_u1_f64(2**53)) == 1
    with localcontext() as ctx:
        ctx.prec = PREC
        ln2 = Decimal(2).ln()
        for K in [1, 2, 3, 2**26, 2**52, 2**52 + 1, 2**53 - 1, 2**53 - 2]:
            exact = Decimal(K).ln() - 53 * ln2
            assert _err_ulps(O.ln_u1_f64(K), exact) <= 1, K
        # powers of two: (j - 53) ln 2 to within one ulp (pins the ln 2 split)
        for j in range(53):
            assert _err_ulps(O.ln_u1_f64(2**j), (j - 53) * ln2) <= 1, j


def test_ln_u1_every_binade(O):
    rng = np.random.default_rng(31)
    Ks = []
    for b in range(54):
        lo, hi = 2**b, min(2**(b + 1), 2**53 + 1)
        Ks += [int(v) for v in rng.integers(lo, hi, 60, dtype=np.uint64)]
    # around sqrt(2) in every binade, where the mantissa is halved
    for b in range(1, 53):
        t = int(math.sqrt(2) * 2**b)
        Ks += [t - 1, t, t + 1]
    Ks += [2**53 - d for d in range(1, 50)]
    got = O.ln_u1_f64_n(np.array(Ks, np.uint64))
    worst = Fraction(0)
    with localcontext() as ctx:
        ctx.prec = PREC
        ln2 = Decimal(2).ln()
        for K, g in zip(Ks, got):
            worst = max(worst, _err_ulps(float(g), Decimal(K).ln() - 53 * ln2))
    assert worst <= 2, float(worst)


def test_sincos_quarter_turns_exact(O):
    want = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    for j in range(4):
        assert O.sincos_turn_f64(j * 2**51) == want[j], j


def test_sincos_against_decimal(O, PI):
    rng = np.random.default_rng(32)
    ks = [int(v) for v in rng.integers(0, 2**53, 1500, dtype=np.uint64)]
    ks += [int(2**e) for e in rng.uniform(0, 53, 400)]            # small angles, every binade
    for j in range(4):
        for d in (1, 2, 1000, 2**20, 2**40):
            ks += [(j * 2**51 + d) % 2**53, (j * 2**51 - d) % 2**53]  # near quarter turns
    ks += [2**50, 3 * 2**50, 5 * 2**50, 7 * 2**50, 2**50 - 1, 2**50 + 1, 2**53 - 1]
    c, s = O.sincos_turn_f64_n(np.array(ks, np.uint64))
    worst = Fraction(0)
    with localcontext() as ctx:
        ctx.prec = PREC
        for k, gc, gs in zip(ks, c, s):
            ec, es = _cos_sin(2 * PI * Decimal(k) / Decimal(2**53))
            worst = max(worst, _err_ulps(float(gc), ec), _err_ulps(float(gs), es))
    assert worst <= 2, float(worst)


def test_normal_pair_against_decimal(O, PI):
    rng = np.random.default_rng(33)
    words = rng.integers(0, 2**32, (600, 4), dtype=np.uint64).tolist()
    words += [[0xFFFFFFFF, 0xFFFFFFFF, 0, 0], [0, 0, 0, 0], [0, 0, 0xFFFFFFFF, 0xFFFFFFFF],
              [0x7FF, 0, 0x800, 0x40000000]]
    with localcontext() as ctx:
        ctx.prec = PREC
        for w0, w1, w2, w3 in words:
            z0, z1 = O.normal_pair_f64(w0, w1, w2, w3)
            x, y = (w1 << 32) | w0, (w3 << 32) | w2
            u1 = Decimal((x >> 11) + 1) / Decimal(2**53)
            R = (-2 * u1.ln()).sqrt() if u1 < 1 else Decimal(0)
            ec, es = _cos_sin(2 * PI * Decimal(y >> 11) / Decimal(2**53))
            bound = 8 * _ulp(R) if R else 0.0
            assert abs(Fraction(z0) - Fraction(R * ec)) <= Fraction(bound), (w0, w1, w2, w3)
            assert abs(Fraction(z1) - Fraction(R * es)) <= Fraction(bound), (w0, w1, w2, w3)
    # u1 = 1: R = +0, both members +0 or -0 by the sign of cos, sin
    z0, z1 = O.normal_pair_f64(0xFFFFFFFF, 0xFFFFFFFF, 0, 0)
    assert (z0, z1) == (0.0, 0.0) and math.copysign(1, z0) == 1


@pytest.mark.parametrize("gen", range(10))
def test_f64_normal_layout(O, gen):
    """Sample p is member p mod 2 of the pair made from words 4(p/2)..4(p/2)+3."""
    seed, ctr, off, n = 0xABCDEF, 3, 1001, 3001
    w = O.fill(gen, O.U32, seed, ctr, 4 * (off // 2), 4 * ((off + n + 1) // 2 - off // 2))
    got = O.fill(gen, O.F64_NORMAL, seed, ctr, off, n)
    for j in list(range(0, n, 37)) + [n - 1]:
        p = off + j
        q = 4 * (p // 2 - off // 2)
        pair = O.normal_pair_f64(w[q], w[q + 1], w[q + 2], w[q + 3])
        assert got[j] == pair[p & 1], (gen, j)
    multi = O.fill_multi(gen, O.F64_NORMAL, seed, ctr, 4, 7, 99).reshape(4, 99)
    for i in range(4):
        assert np.array_equal(multi[i], O.fill(gen, O.F64_NORMAL, seed, ctr + i, 7, 99))
    at = O.samples_at(gen, O.F64_NORMAL, seed, np.full(3, ctr, np.uint32),
                      np.array([off, off + 1, off + 77], np.uint64))
    assert np.array_equal(at, got[[0, 1, 77]])
    last = O.fill(gen, O.F64_NORMAL, seed, ctr, 2**31 - 2, 2)
    w = O.fill(gen, O.U32, seed, ctr, 2**32 - 4, 4)
    assert tuple(last) == O.normal_pair_f64(*w)
    with pytest.raises(ValueError):
        O.fill(gen, O.F64_NORMAL, seed, ctr, 2**31 - 1, 2)


@pytest.mark.parametrize("gen", [0, 3, 4])
def test_f64_normal_statistics(O, gen):
    from scipy import stats
    z = O.fill(gen, O.F64_NORMAL, 2024, 1, 0, 1 << 20)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(stats.skew(z)) < 5 * math.sqrt(6 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / math.sqrt(n / 2)
