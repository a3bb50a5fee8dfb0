"""The oracle's parallel micro-streams (section 5.2's parallel-stream shape):
layout against per-stream fills, the textbook Tyche instance for short
micro-streams, argument ranges, and statistical checks of the concatenated
stream of 16,000 particles x 3 draws across iterations (neighbouring
particles, successive iterations, byte frequencies)."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("gen", range(5))
def test_layout_is_concatenated_micro_streams(O, gen):
    P, D, T, seed0, ctr0 = 37, 5, 4, 2**40 + 3, 1000
    out = O.particle_streams(gen, seed0, P, D, ctr0, T).reshape(T, P, D)
    for t in range(T):
        for p in range(P):
            ref = O.fill(gen, O.U32, seed0 + p, ctr0 + t, 0, D)
            assert np.array_equal(out[t, p], ref), (t, p)


def test_tyche_micro_stream_is_the_textbook_instance(O):
    """Three draws of a Tyche micro-stream are the first three outputs of the
    instance seeded with (particle, iteration)."""
    out = O.particle_streams(4, 500, 10, 3, 7, 2).reshape(2, 10, 3)
    for t in range(2):
        for p in range(10):
            assert list(out[t, p]) == O.tyche_stream(500 + p, 0, 7 + t, 3), (t, p)


def test_ranges(O):
    O.particle_streams(0, 0, 2, 16, 2**32 - 1, 1)
    for args in [(0, 0, 2, 17, 0, 1), (0, 0, 2, 0, 0, 1), (10, 0, 2, 3, 0, 1)]:
        with pytest.raises(ValueError):
            O.particle_streams(*args)
    with pytest.raises(ValueError):
        O.particle_streams(0, 0, 2, 3, 2**32 - 1, 2)
    with pytest.raises(ValueError):
        O.particle_streams(0, 2**64 - 1, 2, 3, 0, 1)


@pytest.mark.parametrize("gen", range(5))
def test_parallel_stream_statistics(O, gen):
    from scipy import stats
    P, D, T = 16000, 3, 6
    w = O.particle_streams(gen, 1, P, D, 1, T)
    u = (w >> 8).astype(np.float64) / 2**24
    m = u.reshape(T, P, D)
    n = P * T
    # neighbouring particles, the same draw
    rho = np.corrcoef(m[:, :-1, 0].ravel(), m[:, 1:, 0].ravel())[0, 1]
    assert abs(rho) < 5 / math.sqrt(n)
    # the same particle in successive iterations
    rho = np.corrcoef(m[:-1, :, 1].ravel(), m[1:, :, 1].ravel())[0, 1]
    assert abs(rho) < 5 / math.sqrt(P * (T - 1))
    # successive draws of one micro-stream
    rho = np.corrcoef(m[:, :, 0].ravel(), m[:, :, 2].ravel())[0, 1]
    assert abs(rho) < 5 / math.sqrt(n)
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    counts = np.bincount(w.view(np.uint8), minlength=256)
    assert stats.chisquare(counts)[1] > 1e-4
