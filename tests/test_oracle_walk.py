"""Pins of the oracle's Brownian walk.

* Each update is one correctly-rounded fused multiply-add: checked step by
  step against exact rational arithmetic rounded once to float32, using the
  oracle's normal fill as the increments (the walk's definition).
* D = 0 leaves every position unchanged.
* Resume: 2k steps equal k steps followed by k more from step0 = k.
* Mean squared displacement from the origin follows 2 * dim * D * t
  (statistical bound from the chi-square law of |x|^2).
"""
import math
from fractions import Fraction

import numpy as np
import pytest


def _round_f32(q: Fraction) -> float:
    """Round a rational to the nearest float32, ties to even (normal range)."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    scale = Fraction(2) ** (23 - e)
    m = a * scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * float(Fraction(fl) / scale)


def test_round_f32_helper():
    for v in [1.0, 0.1, 1 / 3, -2.5e-3, 123456.789]:
        assert _round_f32(Fraction(v)) == float(np.float32(v))


def test_walk_is_fma_of_normal_fill(O):
    seed, ctr0, dim, steps = 31337, 1000, 3, 120
    ids = np.array([0, 5, 77], dtype=np.uint32)
    dt, D = 1e-3, 1.0
    sigma = O.walk_sigma(dt, D)
    assert sigma == float(np.float32(math.sqrt(2 * float(np.float32(D)) * float(np.float32(dt)))))
    pos, _ = O.brownian(seed, ctr0, ids=ids, dim=dim, n_steps=steps, dt=dt, D=D)
    for k, pid in enumerate(ids):
        g = O.fill(0, O.F32_NORMAL, seed, ctr0 + int(pid), 0, dim * steps)
        x = [0.0] * dim
        for s in range(steps):
            for d in range(dim):
                x[d] = _round_f32(Fraction(sigma) * Fraction(float(g[dim * s + d])) + Fraction(x[d]))
        assert [float(v) for v in pos[:, k]] == x


def test_walk_zero_diffusion(O):
    pos, msd = O.brownian(1, 2, n_particles=64, dim=3, n_steps=50, D=0.0, msd_every=10)
    assert not pos.any() and not msd.any()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_walk_resume(O, dim):
    full, _ = O.brownian(5, 6, n_particles=200, dim=dim, n_steps=400)
    half, _ = O.brownian(5, 6, n_particles=200, dim=dim, n_steps=200)
    rest, _ = O.brownian(5, 6, n_particles=200, dim=dim, step0=200, n_steps=200, pos=half)
    assert np.array_equal(full, rest)


def test_walk_ids_select_particles(O):
    full, _ = O.brownian(8, 9, n_particles=100, dim=2, n_steps=30)
    ids = np.array([99, 3, 50], dtype=np.uint32)
    sub, _ = O.brownian(8, 9, ids=ids, dim=2, n_steps=30)
    assert np.array_equal(sub, full[:, ids])


def test_walk_msd_closed_form(O):
    n, dim, steps, every, dt, D = 1 << 14, 3, 1000, 250, 1e-3, 1.0
    pos, msd = O.brownian(2024, 0, n_particles=n, dim=dim, n_steps=steps, dt=dt, D=D,
                          msd_every=every)
    for q, tot in enumerate(msd):
        t = (q + 1) * every * dt
        expect = 2 * dim * D * t
        # |x|^2 = 2Dt * chi2_dim: variance (2Dt)^2 * 2 dim
        se = 2 * D * t * math.sqrt(2 * dim) / math.sqrt(n)
        assert abs(tot / n - expect) < 5 * se, (t, tot / n, expect)
    assert math.isclose(msd[-1], float((pos.astype(np.float64) ** 2).sum()), rel_tol=1e-12)


def test_walk_period_bound(O):
    with pytest.raises(ValueError):
        O.brownian(1, 1, n_particles=1, dim=3, step0=2**32 // 3, n_steps=1)
