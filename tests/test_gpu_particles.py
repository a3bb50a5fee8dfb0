"""GPU parity of the parallel micro-streams (orng_particle_streams) with the
oracle, bit for bit: small cases over every generator and micro-stream
length, a ragged particle count, both schedules (lane per particle; 1,024
slots per workgroup) with their edges, and the section 5.2 shape (16,000
particles x 3 draws) over 2,000 iterations for every generator and over the
measured 22,369 iterations for the store-bound ones, every word."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_19925_amd import orng
    return orng


GUARD = 4 * 1024 * 16  # words after the output: more than a workgroup's share


def _run(R, gen, seed0, P, D, ctr0, T):
    n = T * P * D
    out = torch.full((n + GUARD,), -1, dtype=torch.int32, device="cuda")
    R.orng_particle_streams(gen, seed0, P, D, ctr0, T, out)
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint32)
    assert np.all(host[n:] == 0xFFFFFFFF)  # nothing written past the end
    return host[:n]


@pytest.mark.parametrize("gen", range(10))
@pytest.mark.parametrize("draws", [1, 3, 4, 7, 16])
def test_particle_streams_parity(R, O, gen, draws):
    P, T = 1000, 9
    s0 = 2**40 + 17 if gen != 9 else 2**32 - P  # Philox2x32: seeds up to 2^32 - 1
    got = _run(R, gen, s0, P, draws, 2**32 - T, T)  # ends on the last counter
    ref = O.particle_streams(gen, s0, P, draws, 2**32 - T, T)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("gen", range(10))
def test_particle_streams_paper_shape(R, O, gen):
    """16,000 particles x 3 draws x 2,000 iterations, every word."""
    P, D, T = 16000, 3, 2000
    got = _run(R, gen, 1, P, D, 1, T)
    ref = O.particle_streams(gen, 1, P, D, 1, T)
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, "%d words differ, first at %d" % (bad.size, bad[0])


@pytest.mark.parametrize("gen", range(10))
@pytest.mark.parametrize("draws", [1, 2, 3, 4])
@pytest.mark.parametrize("P,T", [(1024, 5), (1500, 7), (4099, 3)])
def test_particle_streams_flat_schedule(R, O, gen, draws, P, T):
    """Micro-streams of at most four words for 1,024 or more particles (the
    schedule of 1,024 (iteration, particle) slots per workgroup for Philox,
    the Threefry4x32 forms and Squares64; the lane schedule for the others):
    slot ranges that cross iteration rows, a last workgroup with a ragged
    tail, and the last counter."""
    s0 = 2**40 + 5 if gen != 9 else 2**32 - P
    got = _run(R, gen, s0, P, draws, 2**32 - T, T)
    assert np.array_equal(got, O.particle_streams(gen, s0, P, draws, 2**32 - T, T))


@pytest.mark.parametrize("gen", [0, 1, 5, 8])
@pytest.mark.parametrize("shift", [1, 2, 3])
@pytest.mark.parametrize("D", [1, 3, 4])
def test_particle_streams_flat_shape_misaligned(R, O, gen, shift, D):
    """The flat schedule's shape with an output off the 16-byte grid takes the
    lane schedule: same words, nothing written outside the output."""
    P, T = 2048, 4
    n = P * D * T
    buf = torch.full((n + shift + 1,), -1, dtype=torch.int32, device="cuda")
    R.orng_particle_streams(gen, 9, P, D, 3, T, buf.data_ptr() + 4 * shift)
    torch.cuda.synchronize()
    host = buf.cpu().numpy().view(np.uint32)
    assert np.all(host[:shift] == 0xFFFFFFFF) and host[shift + n] == 0xFFFFFFFF
    assert np.array_equal(host[shift:shift + n], O.particle_streams(gen, 9, P, D, 3, T))


@pytest.mark.parametrize("gen", [0, 1, 3, 8])
def test_particle_streams_configured_size(R, O, gen):
    """The measured configuration, 16,000 x 3 x 22,369 words (4 GiB) in one
    launch, compared with the oracle in chunks of 2,000 iterations."""
    P, D, T = 16000, 3, (1 << 30) // 48000
    out = torch.empty(T * P * D, dtype=torch.int32, device="cuda")
    R.orng_particle_streams(gen, 1, P, D, 1, T, out)
    torch.cuda.synchronize()
    for t0 in range(0, T, 2000):
        nt = min(2000, T - t0)
        got = out[t0 * P * D:(t0 + nt) * P * D].cpu().numpy().view(np.uint32)
        ref = O.particle_streams(gen, 1, P, D, 1 + t0, nt)
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, "iterations from %d: %d words differ" % (t0, bad.size)
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("gen", [0, 3, 4, 8, 9])
@pytest.mark.parametrize("shift", [1, 2, 3])
@pytest.mark.parametrize("draws", [1, 3, 5, 16])
def test_particle_streams_misaligned_output(R, O, gen, shift, draws):
    """Outputs 1-3 words off the 16-byte grid (the wave slices are stored in
    16-byte chunks at the output's own phase): same words, nothing written
    before or after the output."""
    P, T = 333, 5
    n = P * draws * T
    buf = torch.full((n + shift + 1,), -1, dtype=torch.int32, device="cuda")
    R.orng_particle_streams(gen, 7, P, draws, 11, T, buf.data_ptr() + 4 * shift)
    torch.cuda.synchronize()
    host = buf.cpu().numpy().view(np.uint32)
    assert np.all(host[:shift] == 0xFFFFFFFF) and host[shift + n] == 0xFFFFFFFF
    assert np.array_equal(host[shift:shift + n], O.particle_streams(gen, 7, P, draws, 11, T))


@pytest.mark.parametrize("P", [2**32 - 1, 2**32 - 1025])
def test_particle_streams_largest_particle_counts(R, O, P):
    """2^32 - 1 particles (the lane schedule, whose workgroup count is rounded
    up without wrapping) and 2^32 - 1025 (the largest count the flat schedule
    takes), one word each for one iteration (16 GiB): the first and last
    1,000 particles against the oracle, nothing written past the end."""
    print("micro-streams P=%d" % P, flush=True)
    out = torch.full((P + 1024,), -1, dtype=torch.int32, device="cuda")
    R.orng_particle_streams(0, 5, P, 1, 3, 1, out)
    torch.cuda.synchronize()
    assert np.all(out[P:].cpu().numpy() == -1)
    for p0 in (0, P - 1000):
        got = out[p0:p0 + 1000].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.particle_streams(0, 5 + p0, 1000, 1, 3, 1)), p0
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("draws", [1, 3, 4])
def test_particle_streams_flat_seeds_across_a_high_word(R, O, draws):
    """Philox4x32 micro-streams on the flat schedule whose seeds seed0 + p
    pass 2^32 inside a workgroup (the carry into the key's high word differs
    between its lanes)."""
    P, T, s0 = 5000, 3, 2**32 - 700
    got = _run(R, 0, s0, P, draws, 11, T)
    assert np.array_equal(got, O.particle_streams(0, s0, P, draws, 11, T))
