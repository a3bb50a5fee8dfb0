"""GPU parity of the float64 fills -- uniforms (ORNG_F64_UNIFORM: sample p
from words 2p and 2p+1) and Box-Muller normals (ORNG_F64_NORMAL: pair m from
words 4m..4m+3, the library's own float64 ln, cos, sin) -- against the oracle,
bit for bit, through every fill path: single stream, many streams, batched and
served requests, with outputs that are 8- but not 16-byte aligned, odd
offsets, ragged tails and the last samples of the stream."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F64, F64N = 3, 4
F64S = (F64, F64N)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_19925_amd import orng
    orng.orng_reset_launch()
    return orng


def _case(R, O, gen, seed, ctr, off, n, pad=0, dist=F64):
    """pad doubles in front of the output: pad odd puts it 8 bytes off the
    16-byte grid."""
    print("case gen=%d dist=%d seed=%d ctr=%d off=%d n=%d pad=%d"
          % (gen, dist, seed, ctr, off, n, pad), flush=True)
    if gen == 9:
        seed &= 0xFFFFFFFF  # Philox2x32 keys with 32 bits
    buf = torch.full((n + pad + 2,), -1, dtype=torch.int64, device="cuda")
    R.orng_fill(gen, dist, seed, ctr, off, n, buf[pad:pad + n])
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    ref = O.fill(gen, dist, seed, ctr, off, n).view(np.int64)
    bad = np.nonzero(host[pad:pad + n] != ref)[0]
    assert bad.size == 0, "first mismatch at %d of %d" % (bad[0], n)
    assert np.all(host[:pad] == -1) and np.all(host[pad + n:] == -1)


@pytest.mark.parametrize("dist", F64S)
@pytest.mark.parametrize("gen", range(10))
def test_f64_fill_parity(R, O, gen, dist):
    n = 3 * 8192 + 2 * 517 + 1
    _case(R, O, gen, 0x0123456789ABCDEF, 7, 0, n, dist=dist)
    _case(R, O, gen, 42, 0, 5, n, dist=dist)                  # odd sample offset
    _case(R, O, gen, 99, 3, 2000, 9001, pad=1, dist=dist)     # output 8 bytes off the 16-byte grid
    _case(R, O, gen, 99, 3, 2001, 9001, pad=1, dist=dist)
    for off, n in [(0, 1), (1, 1), (3, 2), (2**31 - 1, 1), (2**31 - 8193, 8193)]:
        _case(R, O, gen, 5, 6, off, n, dist=dist)


@pytest.mark.parametrize("dist", F64S)
@pytest.mark.parametrize("gen", range(10))
def test_f64_fill_multi(R, O, gen, dist):
    for n_streams, off, per in [(1000, 3, 5), (7, 1, 20001)]:
        out = torch.empty(n_streams * per, dtype=torch.int64, device="cuda")
        R.orng_fill_multi(gen, dist, 11, 100, n_streams, off, per, out)
        torch.cuda.synchronize()
        ref = O.fill_multi(gen, dist, 11, 100, n_streams, off, per).view(np.int64)
        assert np.array_equal(out.cpu().numpy(), ref), (n_streams, off, per)


@pytest.mark.parametrize("dist", F64S)
def test_f64_bulk_sampled(R, O, dist):
    """2^29 doubles (4 GiB) from one stream, checked on sampled positions."""
    n = 1 << 29
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(12)
    for gen in range(10):
        print("bulk gen=%d dist=%d" % (gen, dist), flush=True)
        R.orng_fill(gen, dist, 0xFEED, 1, 0, n, out)
        torch.cuda.synchronize()
        js = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, 200)]))
        got = out[torch.from_numpy(js).cuda()].cpu().numpy()
        ref = O.samples_at(gen, dist, 0xFEED, np.ones(js.size, np.uint32), js.astype(np.uint64))
        assert np.array_equal(got.view(np.int64), ref.view(np.int64)), gen
    del out
    torch.cuda.empty_cache()


def _mixed_requests(rng, m, buf_words):
    rows, off_words = [], 0
    for _ in range(m):
        dist = int(rng.integers(0, 5))
        n = int(2 ** (6 + 12 * rng.random()))
        k = 2 if dist in F64S else 1
        off_words += k - off_words % k  # 8-byte aligned doubles, 4-byte words
        off_words += int(rng.integers(0, 3)) * k
        rows.append(dict(gen=int(rng.integers(0, 10)), dist=dist,
                         seed=int(rng.integers(0, 2**63)), ctr=int(rng.integers(0, 2**32)),
                         offset=int(rng.integers(0, 2**32 // k - n)), n=n, at=off_words))
        if rows[-1]["gen"] == 9:
            rows[-1]["seed"] &= 0xFFFFFFFF  # Philox2x32 keys with 32 bits
        off_words += n * k
    assert off_words < buf_words
    return rows


def _check(O, host_words, rows):
    for q in rows:
        k = 2 if q["dist"] in F64S else 1
        got = host_words[q["at"]:q["at"] + q["n"] * k]
        ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
        assert np.array_equal(got, np.ascontiguousarray(ref).view(np.uint32)), q


def test_f64_in_batched_and_each(R, O):
    rng = np.random.default_rng(13)
    words = 1 << 24
    rows = _mixed_requests(rng, 300, words)
    for fn in (R.orng_fill_batched, R.orng_fill_each):
        buf = torch.full((words,), -1, dtype=torch.int32, device="cuda")
        reqs = R.make_requests([q["gen"] for q in rows], [q["dist"] for q in rows],
                               [q["seed"] for q in rows], [q["ctr"] for q in rows],
                               [q["offset"] for q in rows], [q["n"] for q in rows],
                               buf.data_ptr() + 4 * np.array([q["at"] for q in rows]))
        fn(reqs)
        torch.cuda.synchronize()
        _check(O, buf.cpu().numpy().view(np.uint32), rows)


def test_f64_in_served_mix(R, O):
    rng = np.random.default_rng(14)
    rows = _mixed_requests(rng, 120, 1 << 24)
    arena = torch.empty((64 << 20) // 4, dtype=torch.int32, device="cuda")
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        ts = [R.orng_serve_submit(srv, q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"],
                                  q["n"]) for q in rows]
        for q, t in zip(rows, ts):
            res = R.orng_serve_wait(srv, t)
            k = 2 if q["dist"] in F64S else 1
            off = (res["d_out"] - arena.data_ptr()) // 4
            torch.cuda.synchronize()
            got = arena[off:off + q["n"] * k].cpu().numpy().view(np.uint32)
            ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
            assert np.array_equal(got, np.ascontiguousarray(ref).view(np.uint32)), q
            R.orng_serve_release(srv, t)
    finally:
        R.orng_serve_destroy(srv)


def test_f64_normal_found_anywhere_in_a_large_batch(R, O):
    """The batched launcher picks the kernel variant with the float64 normal
    cases only when a request needs it; its host pass checks the list in
    parallel ranges, so one such request deep in a long list must still be
    found (and the others still served by the same launch)."""
    nreq, per, special = 40000, 16, 33333
    words = nreq * per * 2
    buf = torch.full((words,), -1, dtype=torch.int32, device="cuda")
    base = buf.data_ptr()
    dists = [F64N if i == special else (i % 3) for i in range(nreq)]
    reqs = R.make_requests([i % 9 for i in range(nreq)], dists, [1000 + i for i in range(nreq)],
                           [7] * nreq, [i % 5 for i in range(nreq)], [per] * nreq,
                           base + 8 * per * np.arange(nreq))
    for fn in (R.orng_fill_batched, R.orng_fill_each):
        buf.fill_(-1)
        fn(reqs)
        torch.cuda.synchronize()
        host = buf.cpu().numpy().view(np.uint32).reshape(nreq, 2 * per)
        for i in [0, 1, 2, special - 1, special, special + 1, nreq - 1]:
            k = 2 if dists[i] in F64S else 1
            ref = O.fill(i % 9, dists[i], 1000 + i, 7, i % 5, per)
            assert np.array_equal(host[i, :per * k], np.ascontiguousarray(ref).view(np.uint32)), i
