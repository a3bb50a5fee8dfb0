"""GPU calls whose grids pass one dispatch dimension's limit of 2^32
work-items (64 GiB outputs in one call, which a 288 GB device holds): the
multi-stream fill and integer-range fill cap their grid-strided grids, the
element-wise normal transform, the flat micro-stream schedule and the 2-D
Brownian dynamics launch two-dimensional grids.  Also a whole stream (2^32
words) in one fill, 2^31 integers in one range fill, and whole streams
through the batched, allocation-free batched and served paths.  Sampled
streams at both ends of each output are compared with the oracle, and nothing
is written past the end."""
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


GUARD = 4096


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_fill_multi_beyond_one_grid_dimension(R, O):
    """2^26 + 1000 Philox streams of 256 words: one 1,024-word span each, so
    the uncapped one-wave-per-span grid would be 2^32 + 64,000 work-items."""
    S, L = 2**26 + 1000, 256
    print("fill_multi %d streams x %d words" % (S, L), flush=True)
    out = torch.full((S * L + GUARD,), -1, dtype=torch.int32, device="cuda")
    R.orng_fill_multi(0, 0, 9, 0, S, 0, L, out)
    torch.cuda.synchronize()
    assert np.all(out[S * L:].cpu().numpy() == -1)
    for i0 in (0, 2**25 + 7, S - 50):
        got = out[i0 * L:(i0 + 50) * L].cpu().numpy().view(np.uint32)
        ref = O.fill_multi(0, 0, 9, i0, 50, 0, L).view(np.uint32)
        assert np.array_equal(got, ref), i0
    del out
    _free()


def test_fill_range_beyond_one_grid_dimension(R, O):
    """2^26 + 1000 Philox streams of 256 integers (512 words): one span of
    256 samples each at the built-in shape's 16 groups per span, so the
    capped grid still loops."""
    S, L = 2**26 + 1000, 256
    print("fill_range %d streams x %d samples" % (S, L), flush=True)
    out = torch.full((S * L + GUARD,), -1, dtype=torch.int32, device="cuda")
    R.orng_fill_range(0, 11, 0, S, 0, L, -5, 1000, out)
    torch.cuda.synchronize()
    assert np.all(out[S * L:].cpu().numpy() == -1)
    for i0 in (0, S - 50):
        got = out[i0 * L:(i0 + 50) * L].cpu().numpy()
        assert np.array_equal(got, O.fill_range(0, 11, i0, 50, 0, L, -5, 1000)), i0
    del out
    _free()


def test_normal_pairs_beyond_one_grid_dimension(R, O):
    """2^32 + 1000 pairs (four arrays of 16 GiB): 2^24 + 4 workgroups."""
    n = 2**32 + 1000
    print("normal_pairs n=%d" % n, flush=True)
    x0 = torch.empty(n, dtype=torch.int32, device="cuda")
    x1 = torch.empty(n, dtype=torch.int32, device="cuda")
    # a stream holds 2^32 words: the last 1,000 come from a second stream
    for x, c in ((x0, 1), (x1, 2)):
        R.orng_fill(0, 0, 21, c, 0, 2**32, x)
        R.orng_fill(0, 0, 21, c + 2, 0, n - 2**32, x[2**32:])
    z0 = torch.full((n + GUARD,), -7.0, dtype=torch.float32, device="cuda")
    z1 = torch.full((n + GUARD,), -7.0, dtype=torch.float32, device="cuda")
    R.orng_normal_pairs(x0, x1, n, z0, z1)
    torch.cuda.synchronize()
    assert np.all(z0[n:].cpu().numpy() == -7.0) and np.all(z1[n:].cpu().numpy() == -7.0)
    for i0 in (0, 2**32 - 500, n - 500):
        a = x0[i0:i0 + 500].cpu().numpy().view(np.uint32)
        b = x1[i0:i0 + 500].cpu().numpy().view(np.uint32)
        r0, r1 = O.normal_pair_n(a, b)
        assert np.array_equal(z0[i0:i0 + 500].cpu().numpy().view(np.uint32), r0.view(np.uint32))
        assert np.array_equal(z1[i0:i0 + 500].cpu().numpy().view(np.uint32), r1.view(np.uint32))
    del x0, x1, z0, z1
    _free()


def test_flat_micro_streams_beyond_one_grid_dimension(R, O):
    """2^16 particles x (2^18 + 5) iterations, one word each (64 GiB): the
    flat schedule's 2^24 + 320 workgroups go out as a two-row grid."""
    P, T = 2**16, 2**18 + 5
    n = P * T
    print("particle_streams %d x %d" % (P, T), flush=True)
    out = torch.full((n + GUARD,), -1, dtype=torch.int32, device="cuda")
    R.orng_particle_streams(0, 3, P, 1, 0, T, out)
    torch.cuda.synchronize()
    assert np.all(out[n:].cpu().numpy() == -1)
    for t in (0, 2**18 - 1, T - 1):
        got = out[t * P:(t + 1) * P].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.particle_streams(0, 3, P, 1, t, 1)), t
    del out
    _free()


@pytest.mark.parametrize("gen,dist", [(0, 0), (3, 1), (4, 0), (7, 2), (1, 3), (8, 4)])
def test_whole_stream_in_one_fill(R, O, gen, dist):
    """Every word of one stream in one call (2^32 words: 2^32 float32
    samples, or 2^31 float64 ones; 16 GiB): the first and last 20,000 samples
    against the oracle, nothing written past the end."""
    n = 2**32 if dist < 3 else 2**31
    esz = 4 if dist < 3 else 8
    print("whole stream gen=%d dist=%d n=%d" % (gen, dist, n), flush=True)
    out = torch.full((n * esz // 4 + GUARD,), -1, dtype=torch.int32, device="cuda")
    R.orng_fill(gen, dist, 0x5EED, 7, 0, n, out)
    torch.cuda.synchronize()
    assert np.all(out[n * esz // 4:].cpu().numpy() == -1)
    for s0 in (0, n - 20000):
        w0, w1 = s0 * esz // 4, (s0 + 20000) * esz // 4
        got = out[w0:w1].cpu().numpy().view(np.uint32)
        ref = O.fill(gen, dist, 0x5EED, 7, s0, 20000)
        assert np.array_equal(got, ref.view(np.uint32)), s0
    del out
    _free()


@pytest.mark.parametrize("gen", [0, 4])
def test_whole_stream_of_integers_in_one_fill(R, O, gen):
    """2^31 integers in [lo, hi) (every word pair of one stream, 8 GiB)."""
    n = 2**31
    print("whole-stream range gen=%d" % gen, flush=True)
    out = torch.full((n + GUARD,), -1, dtype=torch.int32, device="cuda")
    R.orng_fill_range(gen, 0x5EED, 7, 1, 0, n, -3, 2**31 - 1, out)
    torch.cuda.synchronize()
    assert np.all(out[n:].cpu().numpy() == -1)
    for s0 in (0, n - 20000):
        got = out[s0:s0 + 20000].cpu().numpy()
        assert np.array_equal(got, O.fill_range(gen, 0x5EED, 7, 1, s0, 20000, -3, 2**31 - 1)), s0
    del out
    _free()


def test_bd2_beyond_one_grid_dimension(R, O):
    """The 2-D Brownian dynamics on 2^31 + 1000 particles (four float64
    arrays, 64 GiB), 3 steps from rest: 2^23 + 4 workgroups as a two-row
    grid; the first and last 1,000 particles against the oracle (particle i
    of a run from pid0 is particle i - i0 of one from pid0 + i0)."""
    n = 2**31 + 1000
    print("bd2 n=%d" % n, flush=True)
    st = torch.zeros((4, n), dtype=torch.float64, device="cuda")
    R.orng_bd2(9, n, 1, 3, 1e-3, 1.0, st[0], st[1], st[2], st[3], 0)
    torch.cuda.synchronize()
    for i0 in (0, n - 1000):
        got = st[:, i0:i0 + 1000].cpu().numpy()
        ref = O.bd2(9 + i0, 1000, step0=1, n_steps=3, dt=1e-3, c=1.0)
        assert np.array_equal(got.view(np.int64), ref.view(np.int64)), i0
    del st
    _free()


@pytest.mark.parametrize("noalloc", [False, True])
def test_batched_whole_streams(R, O, noalloc):
    """One batch of two whole streams: 2^32 Philox words and 2^31 Squares64
    float64 uniforms (16 GiB each), through the batched call and its
    allocation-free form; both ends of each output against the oracle."""
    n0, n1 = 2**32, 2**31
    print("batched whole streams noalloc=%s" % noalloc, flush=True)
    a = torch.full((n0 + GUARD,), -1, dtype=torch.int32, device="cuda")
    b = torch.full((2 * n1 + GUARD,), -1, dtype=torch.int32, device="cuda")
    reqs = R.make_requests([0, 8], [0, 3], [0x5EED, 77], [3, 4], 0, [n0, n1],
                           [a.data_ptr(), b.data_ptr()])
    (R.orng_fill_batched_noalloc if noalloc else R.orng_fill_batched)(reqs)
    torch.cuda.synchronize()
    assert np.all(a[n0:].cpu().numpy() == -1) and np.all(b[2 * n1:].cpu().numpy() == -1)
    for s0 in (0, n0 - 20000):
        got = a[s0:s0 + 20000].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.fill(0, 0, 0x5EED, 3, s0, 20000)), s0
    for s0 in (0, n1 - 20000):
        got = b[2 * s0:2 * (s0 + 20000)].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.fill(8, 3, 77, 4, s0, 20000).view(np.uint32)), s0
    del a, b
    _free()


def test_served_whole_stream(R, O):
    """A served request for a whole stream (2^32 Tyche words, 16 GiB) in a
    17 GiB arena, beside a caller-owned whole stream of 2^31 Threefry4x32
    float64 normals: both ends of each result against the oracle."""
    n0, n1 = 2**32, 2**31
    print("served whole streams", flush=True)
    arena = torch.empty((17 << 30) // 4, dtype=torch.int32, device="cuda")
    mine = torch.full((2 * n1 + GUARD,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the server's streams do not wait for torch's
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        t0 = R.orng_serve_submit(srv, 4, 0, 0x5EED, 6, 0, n0)
        t1 = R.orng_serve_submit(srv, 1, 4, 99, 2, 0, n1, out=mine.data_ptr())
        r0 = R.orng_serve_wait(srv, t0)
        r1 = R.orng_serve_wait(srv, t1)
        assert r0["status"] == 0 and r1["status"] == 0 and r0["n"] == n0 and r1["n"] == n1
        torch.cuda.synchronize()
        off = (r0["d_out"] - arena.data_ptr()) // 4
        for s0 in (0, n0 - 20000):
            got = arena[off + s0:off + s0 + 20000].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, O.fill(4, 0, 0x5EED, 6, s0, 20000)), s0
        assert np.all(mine[2 * n1:].cpu().numpy() == -1)
        for s0 in (0, n1 - 20000):
            got = mine[2 * s0:2 * (s0 + 20000)].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, O.fill(1, 4, 99, 2, s0, 20000).view(np.uint32)), s0
        R.orng_serve_release(srv, t0)
        R.orng_serve_release(srv, t1)
    finally:
        R.orng_serve_destroy(srv)
    del arena, mine
    _free()
