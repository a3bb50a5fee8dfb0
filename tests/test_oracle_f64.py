"""The oracle's float64 uniform fills: sample p is the pinned two-word
conversion of words 2p and 2p+1 of the stream, for every generator, through
every oracle entry point (range fill, direct per-sample evaluation,
multi-stream fill), with positions ending at 2^31."""
import numpy as np
import pytest

F64 = 3


@pytest.mark.parametrize("gen", range(5))
def test_f64_fill_is_word_pairs(O, gen):
    off, n = 12345, 3000
    got = O.fill(gen, F64, 0xABCDEF, 9, off, n)
    assert got.dtype == np.float64
    w = O.fill(gen, 0, 0xABCDEF, 9, 2 * off, 2 * n)
    ref = np.array([O.u01_f64(w[2 * j], w[2 * j + 1]) for j in range(n)])
    assert np.array_equal(got, ref)
    assert got.min() >= 0.0 and got.max() < 1.0


@pytest.mark.parametrize("gen", range(5))
def test_f64_direct_samples_and_multi_stream(O, gen):
    rng = np.random.default_rng(gen)
    pos = rng.integers(0, 2**31, 40).astype(np.uint64)
    pos[:2] = [0, 2**31 - 1]
    ctrs = rng.integers(0, 2**32, 40).astype(np.uint32)
    got = O.samples_at(gen, F64, 77, ctrs, pos)
    for k in range(pos.size):
        ref = O.fill(gen, F64, 77, int(ctrs[k]), int(pos[k]), 1)[0]
        assert got[k] == ref
    multi = O.fill_multi(gen, F64, 5, 100, 3, 17, 50)
    for i in range(3):
        assert np.array_equal(multi[i * 50:(i + 1) * 50], O.fill(gen, F64, 5, 100 + i, 17, 50))


def test_f64_positions_end_at_2_31(O):
    O.fill(0, F64, 1, 1, 2**31 - 4, 4)
    with pytest.raises(ValueError):
        O.fill(0, F64, 1, 1, 2**31 - 4, 5)
    with pytest.raises(ValueError):
        O.fill_multi(0, F64, 1, 1, 2, 2**31, 1)
