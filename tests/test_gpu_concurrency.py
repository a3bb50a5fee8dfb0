"""Several host threads calling the library at once: fills and batched calls
on their own streams, and submitters sharing one server.  Every result must
still equal the oracle bit for bit (the batched path's per-device context
ring and the server's scheduler are the shared state under test)."""
import threading

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


def _threads(fn, n):
    errs = []

    def wrap(i):
        try:
            fn(i)
        except Exception as e:  # reported below, with the thread number
            errs.append((i, repr(e)))

    th = [threading.Thread(target=wrap, args=(i,)) for i in range(n)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs


def test_concurrent_fills_and_batched_calls(R, O):
    n_threads, rounds = 6, 4
    results = {}

    def work(i):
        s = torch.cuda.Stream()
        rng = np.random.default_rng(100 + i)
        with torch.cuda.stream(s):
            for r in range(rounds):
                gen, dist = int(rng.integers(0, 10)), int(rng.integers(0, 3))
                off, n = int(rng.integers(0, 1000)), int(rng.integers(1, 200_000))
                out = torch.empty(n, dtype=torch.int32, device="cuda")
                R.orng_fill(gen, dist, 1000 * i + r, r, off, n, out, s)
                lens = rng.integers(1, 5000, 64)
                pos = np.concatenate([[0], np.cumsum(lens)])
                buf = torch.empty(int(pos[-1]), dtype=torch.int32, device="cuda")
                reqs = R.make_requests(gen, dist, np.arange(64) + 77 * i, r, 0, lens,
                                       buf.data_ptr() + 4 * pos[:-1])
                R.orng_fill_batched(reqs, s)
                s.synchronize()
                results[(i, r)] = (gen, dist, off, n, out.cpu().numpy().view(np.uint32),
                                   lens, pos, buf.cpu().numpy().view(np.uint32))

    _threads(work, n_threads)
    for (i, r), (gen, dist, off, n, got, lens, pos, buf) in results.items():
        ref = O.fill(gen, dist, 1000 * i + r, r, off, n)
        assert np.array_equal(got, np.ascontiguousarray(ref).view(np.uint32)), (i, r)
        for k in range(64):
            ref = O.fill(gen, dist, 77 * i + k, r, 0, int(lens[k]))
            assert np.array_equal(buf[pos[k]:pos[k + 1]],
                                  np.ascontiguousarray(ref).view(np.uint32)), (i, r, k)


def test_concurrent_submitters_share_one_server(R, O):
    arena = torch.empty((64 << 20) // 4, dtype=torch.int32, device="cuda")
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    got = {}

    def work(i):
        rng = np.random.default_rng(200 + i)
        for r in range(30):
            q = dict(gen=int(rng.integers(0, 10)), dist=int(rng.integers(0, 4)),
                     seed=int(rng.integers(0, 2**63)), ctr=int(rng.integers(0, 2**32)),
                     offset=int(rng.integers(0, 2**20)), n=int(rng.integers(1, 100_000)))
            if q["gen"] == 9:
                q["seed"] &= 0xFFFFFFFF  # Philox2x32 keys with 32 bits
            t = R.orng_serve_submit(srv, **q)
            res = R.orng_serve_wait(srv, t)
            k = 2 if q["dist"] == 3 else 1
            off = (res["d_out"] - arena.data_ptr()) // 4
            torch.cuda.synchronize()
            got[(i, r)] = (q, arena[off:off + q["n"] * k].cpu().numpy().view(np.uint32))
            R.orng_serve_release(srv, t)

    try:
        _threads(work, 8)
        st = R.orng_serve_stats(srv)
        assert st["completed"] == 240 and st["released"] == 240 and st["failed"] == 0
    finally:
        R.orng_serve_destroy(srv)
    for (i, r), (q, data) in got.items():
        ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
        assert np.array_equal(data, np.ascontiguousarray(ref).view(np.uint32)), (i, r, q)
