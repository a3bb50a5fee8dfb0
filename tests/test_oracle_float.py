"""Pins of the oracle's float32 conversions against float64 mathematics.

The conversions are this build's readings (the paper gives no float or normal
conversion).  Each is checked exhaustively where its input set is small:
* uniform: all 2^24 top-24-bit parts, exact against float64 arithmetic;
* ln(k 2^-24): all 2^24 arguments, within 2 ulp of float64 log;
* cos/sin(2 pi k 2^-24): all 2^24 arguments, within 1.5 * 2^-24 absolute;
* Box-Muller pair: random word pairs against the float64 formula, within the
  bound that follows from the three bounds above; moments and KS on 10^6.
"""
import math

import numpy as np
import pytest
from scipy import stats


def _ulps(a, ref):
    a = np.asarray(a, np.float64)
    sp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    sp[ref == 0] = float(np.spacing(np.float32(0)))
    return np.abs(a - ref) / sp


def test_u01_exhaustive_top_bits(O):
    top = np.arange(1 << 24, dtype=np.uint32)
    rng = np.random.default_rng(0)
    x = (top << 8) | rng.integers(0, 256, size=top.size, dtype=np.uint32)
    u = O.u01_n(x)
    assert np.array_equal(u.astype(np.float64), top.astype(np.float64) / 2**24)
    assert u.min() == 0.0 and u.max() == np.float32(1 - 2**-24) and u.max() < 1.0


def test_ln_u1_exhaustive(O):
    k = np.arange(1, (1 << 24) + 1, dtype=np.uint32)
    ln = O.ln_u1_n(k)
    ref = np.log(k.astype(np.float64) / 2**24)
    assert ln[-1] == 0.0  # u1 = 1
    assert _ulps(ln, ref).max() <= 2.0
    assert np.all(np.diff(ln.astype(np.float64)) >= 0)  # monotone


def test_sincos2pi_exhaustive(O):
    k = np.arange(1 << 24, dtype=np.uint32)
    c, s = O.sincos2pi_n(k)
    ang = 2 * np.pi * k.astype(np.float64) / 2**24
    assert np.abs(c - np.cos(ang)).max() <= 1.5 * 2**-24
    assert np.abs(s - np.sin(ang)).max() <= 1.5 * 2**-24
    # exact at the quarter turns
    q = np.array([0, 1 << 22, 2 << 22, 3 << 22], dtype=np.uint32)
    cq, sq = O.sincos2pi_n(q)
    assert list(cq) == [1, 0, -1, 0] and list(sq) == [0, 1, 0, -1]


def test_normal_pair_vs_float64_formula(O):
    rng = np.random.default_rng(1)
    n = 1 << 20
    x0 = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    x1 = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    # include the extremes of u1: largest radius (x0 top = 0) and zero radius
    x0[:4] = [0, 255, 0xFFFFFF00, 0xFFFFFFFF]
    z0, z1 = O.normal_pair_n(x0, x1)
    u1 = ((x0 >> 8).astype(np.float64) + 1) / 2**24
    u2 = (x1 >> 8).astype(np.float64) / 2**24
    r = np.sqrt(-2 * np.log(u1))
    e0 = np.abs(z0 - r * np.cos(2 * np.pi * u2))
    e1 = np.abs(z1 - r * np.sin(2 * np.pi * u2))
    # |dR| <= R*(2 ulp of ln)/2 + 0.5 ulp(R) ; |d trig| <= 1.5*2^-24 ; + product rounding
    bound = 4e-7 * np.maximum(r, 1.0)
    assert np.all(e0 <= bound) and np.all(e1 <= bound)
    assert z0[2] == 0.0 or abs(z0[2]) < 1e-3  # u1 = 1 - ... tiny radius
    assert z0[3] == 0.0 and z1[3] == 0.0  # u1 == 1 exactly -> R = 0


def test_normal_moments_and_ks(O):
    z = O.fill(0, O.F32_NORMAL, 2023, 1, 0, 1 << 20).astype(np.float64)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(stats.skew(z)) < 5 * math.sqrt(6 / n)
    assert abs(stats.kurtosis(z)) < 5 * math.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a pair are independent
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / math.sqrt(n / 2)


@pytest.mark.parametrize("gen", range(5))
def test_uniform_ks_all_gens(O, gen):
    u = O.fill(gen, O.F32_UNIFORM, 77, 3, 5, 1 << 18).astype(np.float64)
    assert u.min() >= 0 and u.max() < 1
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_normal_sample_is_pair_member(O):
    # sample p of a normal fill is member p mod 2 of the pair from words 2(p//2), 2(p//2)+1
    for gen in range(5):
        w = O.fill(gen, O.U32, 11, 12, 0, 64)
        z = O.fill(gen, O.F32_NORMAL, 11, 12, 0, 64)
        z0, z1 = O.normal_pair_n(w[0::2], w[1::2])
        assert np.array_equal(z[0::2], z0) and np.array_equal(z[1::2], z1)
        odd = O.fill(gen, O.F32_NORMAL, 11, 12, 7, 9)
        assert np.array_equal(odd.view(np.uint32), z[7:16].view(np.uint32))
