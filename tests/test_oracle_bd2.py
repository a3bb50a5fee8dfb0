"""Pins of the oracle's float64 uniform and of its transcription of the paper's
2-D Brownian dynamics example (section 4, Fig. 1), against exact rational
arithmetic, an exactly solvable special case and the closed-form moments of
the velocity process."""
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def _u_exact(w0, w1):
    x = (int(w1) << 32) | int(w0)
    return Fraction(x >> 11, 1 << 53)


def test_u01_f64_is_the_top_53_bits_exactly(O):
    rng = np.random.default_rng(11)
    words = [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (0x7FF, 0), (0x800, 0), (0, 1),
             (0xFFFFFFFF, 0), (0, 0x80000000)] + \
        [tuple(int(v) for v in rng.integers(0, 2**32, 2)) for _ in range(2000)]
    for w0, w1 in words:
        u = O.u01_f64(w0, w1)
        assert Fraction(u) == _u_exact(w0, w1), (w0, w1)
        assert 0.0 <= u < 1.0
    assert O.u01_f64(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert O.u01_f64(0x7FF, 0) == 0.0 and O.u01_f64(0x800, 0) == 2.0**-53


@pytest.mark.parametrize("pid", [0, 12345, (7 << 32) | 99])
def test_bd2_special_case_kick_only(O, pid):
    """gamma/m = 2^10 with dt = 2^-10 makes the drag remove the whole velocity
    in one step (the decay 1 - c dt is exactly 0), and sqrt(dt) = 2^-5, so
    after every step v equals the kick alone, (2u - 1) / 32, with u from words
    0..3 of Philox stream (pid, step); from rest, x after two steps is exactly
    dt (v1 + v2)."""
    c, dt = 2.0**10, 2.0**-10
    step0 = 17
    st = O.bd2(pid, 1, step0=step0, n_steps=1, dt=dt, c=c,
               state=[[0.0], [0.0], [0.3], [-5.0]])
    w = O.philox4x32_10([0, step0, 0, 0], [pid & 0xFFFFFFFF, pid >> 32])
    v1 = [(2 * _u_exact(w[0], w[1]) - 1) / 32, (2 * _u_exact(w[2], w[3]) - 1) / 32]
    assert Fraction(st[2, 0]) == v1[0] and Fraction(st[3, 0]) == v1[1]
    assert Fraction(st[0, 0]) == v1[0] * Fraction(dt) and Fraction(st[1, 0]) == v1[1] * Fraction(dt)
    st2 = O.bd2(pid, 1, step0=step0 + 1, n_steps=1, dt=dt, c=c, state=st)
    w = O.philox4x32_10([0, step0 + 1, 0, 0], [pid & 0xFFFFFFFF, pid >> 32])
    v2 = [(2 * _u_exact(w[0], w[1]) - 1) / 32, (2 * _u_exact(w[2], w[3]) - 1) / 32]
    assert Fraction(st2[2, 0]) == v2[0] and Fraction(st2[3, 0]) == v2[1]
    assert Fraction(st2[0, 0]) == (v1[0] + v2[0]) * Fraction(dt)
    assert Fraction(st2[1, 0]) == (v1[1] + v2[1]) * Fraction(dt)
    # two steps in one call are the same two steps
    assert np.array_equal(O.bd2(pid, 1, step0=step0, n_steps=2, dt=dt, c=c,
                                state=[[0.0], [0.0], [0.3], [-5.0]]), st2)


def test_bd2_moments_match_the_ar1_closed_form(O):
    """From rest, v_s = a v_(s-1) + k_s with a = 1 - c dt and kicks k uniform on
    [-sqrt(dt), sqrt(dt)) (variance dt/3), so Var v_T = (dt/3)(1 - a^2T)/(1 - a^2);
    x_T = dt * sum v_s has Var x_T = dt^2 sum_(s,t) a^|t-s| Var v_min(s,t).  The
    x and y kicks come from different words, so vx and vy are uncorrelated."""
    n, T, c, dt = 40000, 50, 50.0, 1e-2
    st = O.bd2(1000, n, step0=1, n_steps=T, dt=dt, c=c)
    a = 1.0 - c * dt
    sk2 = dt / 3.0
    var_v = [sk2 * (1 - a ** (2 * s)) / (1 - a * a) for s in range(T + 1)]
    var_x = dt * dt * sum(a ** abs(t - s) * var_v[min(s, t)]
                          for s in range(1, T + 1) for t in range(1, T + 1))
    tol = 5 * np.sqrt(2.0 / n)  # 5 standard errors of a variance estimate
    for comp in (2, 3):
        v = st[comp]
        assert abs(v.mean()) < 5 * np.sqrt(var_v[T] / n)
        assert abs(v.var() / var_v[T] - 1) < tol
    for comp in (0, 1):
        x = st[comp]
        assert abs(x.mean()) < 5 * np.sqrt(var_x / n)
        assert abs(x.var() / var_x - 1) < tol
    assert abs(np.corrcoef(st[2], st[3])[0, 1]) < 5 / np.sqrt(n)


def test_bd2_subset_and_ranges(O):
    full = O.bd2(77, 10, step0=3, n_steps=6)
    sub = O.bd2(77, ids=[3, 7], step0=3, n_steps=6)
    assert np.array_equal(sub, full[:, [3, 7]])
    O.bd2(5, 2, step0=2**32 - 1, n_steps=1)  # the last counter
    with pytest.raises(ValueError):
        O.bd2(5, 2, step0=2**32 - 1, n_steps=2)
