"""The allocation-free batched call (orng_fill_batched_noalloc) against
orng_fill_batched, through the C ABI: the same request lists give the same
output words, guard words included, on consecutive calls whose batches shrink
(the second and third calls reuse the library's fixed device array after a
larger batch), and the limits are rejected before anything is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_19925_amd import orng
    orng.orng_reset_launch()
    return orng


def _mixed_batch(rng, m, max_log2=14):
    """Requests over every generator and distribution, lengths log-uniform,
    a few empty ones; outputs packed with one guard word after each request,
    float64 requests on 8-byte boundaries, the rest at any word."""
    L = np.maximum(1, np.floor(2.0 ** (max_log2 * rng.random(m)))).astype(np.int64)
    L[rng.choice(m, max(1, m // 50), replace=False)] = 0
    gen = rng.integers(0, 10, m)
    dist = rng.integers(0, 5, m)
    k = np.where(dist >= 3, 2, 1)
    seed = rng.integers(0, 2**63, m, dtype=np.int64).astype(np.uint64) * 2 + 1
    seed = np.where(gen == 9, seed & np.uint64(0xFFFFFFFF), seed)  # Philox2x32: 32-bit keys
    ctr = rng.integers(0, 2**32, m, dtype=np.uint64)
    lim = np.where(k == 2, 2**31, 2**32)
    off = np.floor(rng.random(m) * (lim - L + 1)).astype(np.uint64)
    starts = np.zeros(m, np.int64)
    pos = 1
    for i in range(m):
        if k[i] == 2:
            pos += pos & 1
        starts[i] = pos
        pos += int(L[i] * k[i]) + 1
    return gen, dist, seed, ctr, off, L, starts, pos + 2


def _both(R, batch):
    gen, dist, seed, ctr, off, L, starts, words = batch
    outs = []
    for fn in (R.orng_fill_batched, R.orng_fill_batched_noalloc):
        buf = torch.full((words,), -1, dtype=torch.int32, device="cuda")
        reqs = R.make_requests(gen, dist, seed, ctr, off, L, buf.data_ptr() + 4 * starts)
        fn(reqs)
        outs.append(buf)
    torch.cuda.synchronize()
    return outs


def test_noalloc_equals_batched_on_shrinking_calls(R, O):
    # call 1: the 10^5 uneven Philox streams of the batched workload
    from paper_2310_19925_amd import inputs
    b = inputs.batched_requests()
    total = int(b["out_off"][-1])
    print("noalloc call 1: 10^5 Philox u32 requests,", total, "words", flush=True)
    outs = []
    for fn in (R.orng_fill_batched, R.orng_fill_batched_noalloc):
        buf = torch.full((total + 1,), -1, dtype=torch.int32, device="cuda")
        reqs = R.make_requests(0, 0, b["seed"], b["ctr"], b["offset"], b["n"],
                               buf.data_ptr() + 4 * b["out_off"][:-1])
        fn(reqs)
        outs.append(buf)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    assert int(outs[1][-1]) == -1
    got = outs[1][: int(b["n"][0])].cpu().numpy().view(np.uint32)
    ref = O.fill(0, 0, int(b["seed"][0]), int(b["ctr"][0]), int(b["offset"][0]), int(b["n"][0]))
    assert np.array_equal(got, ref.view(np.uint32))
    del outs, buf
    torch.cuda.empty_cache()

    # calls 2 and 3: smaller batches mixing every generator and distribution
    rng = np.random.default_rng(11)
    for m in (600, 37):
        print("noalloc call: mixed batch of", m, "requests", flush=True)
        batch = _mixed_batch(rng, m)
        a, c = _both(R, batch)
        assert torch.equal(a, c), ("batch of", m)
        gen, dist, seed, ctr, off, L, starts, _ = batch
        host = c.cpu().numpy().view(np.uint32)
        for i in rng.choice(m, 12, replace=False):
            k = 2 if dist[i] >= 3 else 1
            got = host[starts[i]: starts[i] + L[i] * k]
            ref = O.fill(int(gen[i]), int(dist[i]), int(seed[i]), int(ctr[i]), int(off[i]),
                         int(L[i]))
            assert np.array_equal(got, ref.view(np.uint32)), ("request", i)


def test_noalloc_limits(R):
    buf = torch.full((1 << 20,), -1, dtype=torch.int32, device="cuda")
    # more requests than the fixed table holds (all empty: validation passes)
    many = R.make_requests(0, 0, 1, 1, 0, np.zeros(R.NOALLOC_MAX_REQUESTS + 1, np.int64), 0)
    with pytest.raises(R.OrngError) as e:
        R.orng_fill_batched_noalloc(many)
    assert e.value.status == R.ENOMEM
    # more tiles than the fixed tile map holds: every request aims at the same
    # (real) buffer, so nothing out of bounds could be written even if the
    # check failed
    m = R.NOALLOC_MAX_REQUESTS
    big = R.make_requests(0, 0, 1, 1, 0, np.full(m, 1 << 20, np.int64), buf.data_ptr())
    big["n"][:] = 1 << 20
    with pytest.raises(R.OrngError) as e:
        R.orng_fill_batched_noalloc(big)
    assert e.value.status == R.ENOMEM
    torch.cuda.synchronize()
    assert bool((buf == -1).all()), "a rejected batch wrote output"
    # errors of the requests themselves come first
    bad = R.make_requests([0, 10], 0, 1, 1, 0, 16, buf.data_ptr())
    with pytest.raises(R.OrngError) as e:
        R.orng_fill_batched_noalloc(bad)
    assert e.value.status == R.EINVAL
    R.orng_fill_batched_noalloc(R.make_requests(0, 0, 1, 1, 0, 0, 0))  # nothing to do
