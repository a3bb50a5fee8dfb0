"""GPU parity of the fill paths against the oracle (bit-exact, every generator
and distribution), through the C-ABI.

Small cases are compared element by element: they span several spans/tiles
and end in a ragged tail.  A sweep with the grid capped at 1 and 7
workgroups makes every kernel loop over many spans and is compared element
by element.  The configured 2^30-sample bulk fills are compared element by
element in chunks of 2^26 samples, and on sampled positions (the oracle
evaluates each one directly) together with properties that hold at any size.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GENS = range(10)
DISTS = range(3)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_19925_amd import orng
    orng.orng_reset_launch()
    return orng


def as_u32(t):
    return t.cpu().numpy().view(np.uint32)


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def key32(gen, seed):
    """Philox2x32-10 (generator 9) takes seeds below 2^32: its tests use the
    low word of the seed the other generators take."""
    return seed & 0xFFFFFFFF if gen == 9 else seed


def _case(R, O, gen, dist, seed, ctr, off, n, pad=0):
    """Fill through the C-ABI into a buffer starting `pad` words into an
    allocation (pad != 0 makes the output misaligned w.r.t. 16 bytes)."""
    print("case gen=%d dist=%d seed=%d ctr=%d off=%d n=%d pad=%d" % (gen, dist, seed, ctr, off, n,
                                                                    pad), flush=True)
    seed = key32(gen, seed)
    buf = torch.full((n + pad + 4,), -1, dtype=torch.int32, device="cuda")
    out = buf[pad:pad + n]
    R.orng_fill(gen, dist, seed, ctr, off, n, out)
    torch.cuda.synchronize()
    got = as_u32(out)
    ref = bits(O.fill(gen, dist, seed, ctr, off, n))
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, "first mismatch at %d of %d" % (bad[0], n)
    # nothing written outside [pad, pad + n)
    rest = as_u32(buf)
    assert np.all(rest[:pad] == 0xFFFFFFFF) and np.all(rest[pad + n:] == 0xFFFFFFFF)


@pytest.mark.parametrize("gen", GENS)
@pytest.mark.parametrize("dist", DISTS)
def test_fill_parity_small(R, O, gen, dist):
    n = 3 * 16384 + 4 * 517 + 3  # several tiles/spans + ragged tail
    _case(R, O, gen, dist, 0x0123456789ABCDEF, 7, 0, n)
    _case(R, O, gen, dist, 42, 0, 5, n)               # odd offset: pairs split
    _case(R, O, gen, dist, 2**64 - 1, 2**32 - 1, 16381, 40000)


@pytest.mark.parametrize("gen", GENS)
@pytest.mark.parametrize("pad", [1, 2, 3])
def test_fill_parity_misaligned(R, O, gen, pad):
    for dist in DISTS:
        _case(R, O, gen, dist, 99 + pad, 3, 4 * 1000, 9001, pad=pad)
        _case(R, O, gen, dist, 99 + pad, 3, 4 * 1000 + pad, 9001, pad=pad)  # realigned


@pytest.mark.parametrize("gen", GENS)
def test_fill_tiny_and_edges(R, O, gen):
    for dist in DISTS:
        for off, n in [(0, 1), (1, 1), (3, 2), (0, 3), (0, 5), (63, 65), (2**32 - 1, 1),
                       (2**32 - 7, 7), (2**32 - 16384 * 2 - 5, 16384 * 2 + 5)]:
            _case(R, O, gen, dist, 5, 6, off, n)


def test_fill_errors(R):
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(R.OrngError) as e:
        R.orng_fill(10, 0, 1, 1, 0, 4, out)
    assert e.value.status == R.EINVAL
    with pytest.raises(R.OrngError) as e:
        R.orng_fill(9, 0, 2**32, 1, 0, 4, out)  # Philox2x32 keys with 32 bits
    assert e.value.status == R.EINVAL
    R.orng_fill(9, 0, 2**32 - 1, 1, 0, 4, out)
    with pytest.raises(R.OrngError) as e:
        R.orng_fill(0, 5, 1, 1, 0, 4, out)
    assert e.value.status == R.EINVAL
    with pytest.raises(R.OrngError) as e:
        R.orng_fill(0, 0, 1, 1, 2**32 - 3, 4, out)
    assert e.value.status == R.ERANGE
    with pytest.raises(R.OrngError) as e:
        R.orng_fill(0, 0, 1, 1, 0, 4, out.data_ptr() + 2)
    assert e.value.status == R.EINVAL
    with pytest.raises(R.OrngError) as e:
        R.orng_fill(0, 0, 1, 1, 0, 4, 0)
    assert e.value.status == R.EINVAL
    R.orng_fill(0, 0, 1, 1, 2**32, 0, 0)  # n == 0 is a no-op
    with pytest.raises(R.OrngError) as e:
        R.orng_fill_multi(0, 0, 1, 2**32 - 2, 3, 0, 4, out)
    assert e.value.status == R.ERANGE


def test_plain_multistream_config(R, O):
    """Seed 42, 2^20 streams (counters 0..2^20-1) x 4 words, u32 and f32
    uniform: compared in full."""
    for dist in (0, 1):
        out = R.fill_multi(0, dist, 42, 0, 1 << 20, 0, 4)
        torch.cuda.synchronize()
        ref = O.fill_multi(0, dist, 42, 0, 1 << 20, 0, 4)
        assert np.array_equal(as_u32(out), bits(ref))


@pytest.mark.parametrize("gen", GENS)
@pytest.mark.parametrize("dist", DISTS)
def test_fill_multi_parity(R, O, gen, dist):
    for n_streams, off, per in [(1000, 0, 4), (333, 3, 9), (50, 100, 1000), (3, 0, 40000),
                                (70, 16380, 70)]:
        out = R.fill_multi(gen, dist, 1234, 2**32 - n_streams, n_streams, off, per)
        torch.cuda.synchronize()
        ref = O.fill_multi(gen, dist, 1234, 2**32 - n_streams, n_streams, off, per)
        assert np.array_equal(as_u32(out), bits(ref)), (n_streams, off, per)


@pytest.mark.parametrize("gen", [0, 3, 4, 9])
def test_launch_geometry_invariance(R, O, gen):
    """Results do not depend on workgroup size, span length, grid size or
    store kind (paper section 4: unique streams regardless of thread count)."""
    n, off = 5 * 16384 + 11, 9
    ref = bits(O.fill(gen, 2, 77, 8, off, n))
    try:
        for wg, un, mx, nt in [(64, 1, 1, 2), (128, 2, 3, 1), (256, 4, 0, 1), (512, 16, 7, 2),
                               (192, 64, 0, 2), (320, 3, 2, 1)]:
            R.orng_set_launch(wg, un, mx, nt)
            out = R.fill(gen, 2, 77, 8, off, n)
            torch.cuda.synchronize()
            assert np.array_equal(as_u32(out), ref), (wg, un, mx, nt)
    finally:
        R.orng_reset_launch()


def test_bulk_config_sampled(R, O):
    """2^30 samples per generator and distribution, single stream, seed from
    PCG64: sampled positions against the oracle, plus chunk invariance."""
    from paper_2310_19925_amd import inputs
    seed = inputs.bulk_seed()
    n = inputs.BULK_N
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(7)
    pos = np.concatenate([rng.integers(0, n, 3000), [0, 1, 2, 3, n - 4, n - 3, n - 2, n - 1],
                          16384 * np.arange(1, 40)]).astype(np.int64)
    idx = torch.from_numpy(pos).cuda()
    for gen in GENS:
        seed = key32(gen, inputs.bulk_seed())
        for dist in DISTS:
            print("bulk gen=%d dist=%d" % (gen, dist), flush=True)
            R.orng_fill(gen, dist, seed, 0, 0, n, out)
            got = as_u32(out[idx])
            ref = bits(O.samples_at(gen, dist, seed, np.zeros(pos.size, np.uint32), pos))
            assert np.array_equal(got, ref), (gen, dist)
            # a chunk starting at an odd offset equals the matching slice
            part = R.fill(gen, dist, seed, 0, 12345677, 1 << 20).view(torch.int32)
            assert torch.equal(part, out[12345677:12345677 + (1 << 20)])
            if dist == 1:
                f = out.view(torch.float32)
                assert float(f.min()) >= 0.0 and float(f.max()) < 1.0
            if dist == 2:
                f = out.view(torch.float32)[: 1 << 26].double()
                assert abs(float(f.mean())) < 5 / 2**13 and abs(float(f.var()) - 1) < 5 * 2**-12.5
    del out
    torch.cuda.empty_cache()


def test_normal_transform_exhaustive(R, O):
    """Every argument of the logarithm (all 2^24 values of x0 >> 8) and of the
    quarter-turn sine/cosine (all 2^24 values of x1 >> 8) through the GPU
    Box-Muller transform, bit-exact against the oracle.  With x1 = 0 the cosine
    is exactly 1, so z0 is the radius itself: this pins the division and the
    square root of the GPU path to IEEE results on their whole input set."""
    k = torch.arange(1 << 24, dtype=torch.int64, device="cuda")
    z0 = torch.empty(1 << 24, dtype=torch.float32, device="cuda")
    z1 = torch.empty_like(z0)
    words = (k << 8).to(torch.int32)
    low = torch.full_like(words, 0x5A)
    cases = [(words | low, torch.zeros_like(words)),             # every u1, cos = 1
             (torch.full_like(words, 0x12345678), words | low),  # every u2, radius A
             (torch.full_like(words, 0x00ABCDEF), words)]        # every u2, radius B
    for x0, x1 in cases:
        R.orng_normal_pairs(x0, x1, 1 << 24, z0, z1)
        torch.cuda.synchronize()
        a0, a1 = O.normal_pair_n(x0.cpu().numpy().view(np.uint32), x1.cpu().numpy().view(np.uint32))
        g0, g1 = as_u32(z0), as_u32(z1)
        bad = np.nonzero((g0 != a0.view(np.uint32)) | (g1 != a1.view(np.uint32)))[0]
        assert bad.size == 0, "mismatch at %d of 2^24" % bad[0]


def test_normal_pairs_errors(R):
    t = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(R.OrngError) as e:
        R.orng_normal_pairs(t, 0, 8, t, t)
    assert e.value.status == R.EINVAL
    R.orng_normal_pairs(0, 0, 0, 0, 0)


@pytest.mark.parametrize("gen", range(5))
def test_bulk_config_elementwise(R, O, gen):
    """The configured bulk fills -- 2^30 samples of one stream (seed drawn from
    PCG64, counter 0) as uint32, float32 uniform and float32 normal -- in the
    launch configuration the benchmark times, compared with the oracle element
    by element in chunks of 2^26 samples."""
    from paper_2310_19925_amd import inputs
    seed = inputs.bulk_seed()
    n, ch = inputs.BULK_N, 1 << 26
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    host = torch.empty(ch, dtype=torch.int32, pin_memory=True)
    try:
        for dist in DISTS:
            print("bulk elementwise gen=%d dist=%d" % (gen, dist), flush=True)
            R.orng_fill(gen, dist, seed, 0, 0, n, out)
            for c in range(0, n, ch):
                host.copy_(out[c:c + ch])
                got = host.numpy().view(np.uint32)
                ref = bits(O.fill(gen, dist, seed, 0, c, ch))
                if not np.array_equal(got, ref):
                    bad = np.nonzero(got != ref)[0]
                    pytest.fail("gen %d dist %d: %d mismatches, first at sample %d"
                                % (gen, dist, bad.size, c + bad[0]))
    finally:
        del out
        torch.cuda.empty_cache()


@pytest.mark.parametrize("gen", GENS)
def test_grid_stride_sweep(R, O, gen):
    """The grid capped at 1 and at 7 workgroups, so that every wave of every
    fill kernel loops over many spans (or Tyche tiles): each of the five
    distributions from an odd offset into an output off the 16-byte grid, and
    a multi-stream fill whose waves cross stream boundaries, element by
    element against the oracle."""
    seed = key32(gen, 0x9E3779B97F4A7C15)
    n = (1 << 20) + 2333
    try:
        for cap in (1, 7):
            R.orng_set_launch(max_wgs=cap)
            for dist in range(5):
                k = 2 if dist >= 3 else 1
                pad = 2 if k == 2 else 1
                print("sweep gen=%d dist=%d cap=%d" % (gen, dist, cap), flush=True)
                buf = torch.full((n * k + pad + 4,), -1, dtype=torch.int32, device="cuda")
                out = buf[pad:pad + n * k]
                R.orng_fill(gen, dist, seed, 5, 3, n, out)
                torch.cuda.synchronize()
                got = as_u32(buf)
                ref = bits(O.fill(gen, dist, seed, 5, 3, n))
                assert np.array_equal(got[pad:pad + n * k], ref), (gen, dist, cap)
                assert np.all(got[:pad] == 0xFFFFFFFF) and np.all(got[pad + n * k:] == 0xFFFFFFFF)
            per, ns = 20011, 37
            m = torch.full((ns * per,), -1, dtype=torch.int32, device="cuda")
            R.orng_fill_multi(gen, 2, seed, 9, ns, 11, per, m)
            torch.cuda.synchronize()
            ref = bits(O.fill_multi(gen, 2, seed, 9, ns, 11, per))
            assert np.array_equal(as_u32(m), ref), (gen, "multi", cap)
    finally:
        R.orng_reset_launch()


@pytest.mark.parametrize("gen", range(10))
def test_aligned_interior_spans_sweep(R, O, gen):
    """Outputs on the block grid from block-aligned offsets, so that every span
    but the first and last is wholly inside the range (the fill kernel's
    check-free loop where it is compiled in): each distribution under the
    tuned launch and with the grid capped at 1 and 7 workgroups (every wave
    loops over many such spans), and a multi-stream fill of 37 aligned
    streams, element by element against the oracle, with nothing written
    around the output."""
    seed = key32(gen, 0xD1B54A32D192ED03)
    n = (1 << 20) + 4 * 777
    try:
        for cap in (0, 1, 7):
            R.orng_set_launch(max_wgs=cap)
            for dist in range(5):
                k = 2 if dist >= 3 else 1
                off = 16384 * 3 + 4 * 5 if k == 1 else 8192 * 3 + 2 * 5  # block-aligned
                print("aligned gen=%d dist=%d cap=%d" % (gen, dist, cap), flush=True)
                buf = torch.full((n * k + 8,), -1, dtype=torch.int32, device="cuda")
                out = buf[4:4 + n * k]
                assert out.data_ptr() % 16 == 0
                R.orng_fill(gen, dist, seed, 12, off, n, out)
                torch.cuda.synchronize()
                got = as_u32(buf)
                ref = bits(O.fill(gen, dist, seed, 12, off, n))
                assert np.array_equal(got[4:4 + n * k], ref), (gen, dist, cap)
                assert np.all(got[:4] == 0xFFFFFFFF) and np.all(got[4 + n * k:] == 0xFFFFFFFF)
            per, ns = 20480, 37
            m = torch.full((ns * per,), -1, dtype=torch.int32, device="cuda")
            R.orng_fill_multi(gen, 1, seed, 9, ns, 4096, per, m)
            torch.cuda.synchronize()
            ref = bits(O.fill_multi(gen, 1, seed, 9, ns, 4096, per))
            assert np.array_equal(as_u32(m), ref), (gen, "multi", cap)
    finally:
        R.orng_reset_launch()


def test_squares_seed_pair_shares_streams(R, O):
    """The one pair of 32-bit seeds with the same Squares key (the key map is
    two-to-one) gives the same Squares32 and Squares64 words on the GPU."""
    a, b = 369106595, 2888123536
    for gen in (3, 8):
        x = R.fill(gen, 0, a, 5, 1, 10001)
        y = R.fill(gen, 0, b, 5, 1, 10001)
        torch.cuda.synchronize()
        assert torch.equal(x, y)
        assert np.array_equal(x.cpu().numpy().view(np.uint32), O.fill(gen, 0, b, 5, 1, 10001))
