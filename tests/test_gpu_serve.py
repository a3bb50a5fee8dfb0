"""GPU tests of the continuous-batching server: every result equals the oracle
(and the same request served alone), admission respects the HBM budget, and
the ticket life cycle and error codes behave as documented."""
import time

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


def _arena(nbytes):
    return torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")


def _read(arena, res):
    off = (res["d_out"] - arena.data_ptr()) // 4
    torch.cuda.synchronize()
    return arena[off:off + res["n"]].cpu().numpy().view(np.uint32)


def _random_reqs(rng, m, lo=10, hi=16):
    out = []
    for _ in range(m):
        n = int(2 ** (lo + (hi - lo) * rng.random()))
        out.append(dict(gen=int(rng.integers(0, 10)), dist=int(rng.integers(0, 3)),
                        seed=int(rng.integers(0, 2**63)), ctr=int(rng.integers(0, 2**32)),
                        offset=int(rng.integers(0, 2**32 - n)), n=n))
        if out[-1]["gen"] == 9:
            out[-1]["seed"] &= 0xFFFFFFFF  # Philox2x32 keys with 32 bits
    return out


def test_serve_mixed_parity(R, O):
    rng = np.random.default_rng(1)
    arena = _arena(64 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        reqs = _random_reqs(rng, 80)
        tickets = [R.orng_serve_submit(srv, **q) for q in reqs]
        for q, t in zip(reqs, tickets):
            res = R.orng_serve_wait(srv, t)
            assert res["status"] == 0 and res["n"] == q["n"]
            assert res["t_submit_ns"] <= res["t_admit_ns"] <= res["t_done_ns"]
            ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
            assert np.array_equal(_read(arena, res), ref.view(np.uint32)), q
            R.orng_serve_release(srv, t)
        st = R.orng_serve_stats(srv)
        assert st["completed"] == 80 and st["released"] == 80 and st["failed"] == 0
        assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"]
    finally:
        R.orng_serve_destroy(srv)


def test_serve_caller_outputs_and_small_steps(R, O):
    """Caller buffers (misaligned), and a step size far below the request
    sizes so every request spans many steps mixed with the others."""
    rng = np.random.default_rng(2)
    arena = _arena(1 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena, step_words=8192)
    try:
        reqs = _random_reqs(rng, 20, 12, 15)
        bufs, tickets = [], []
        for q in reqs:
            b = torch.full((q["n"] + 2,), -1, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()  # the server's streams do not wait for torch's
            bufs.append(b)
            tickets.append(R.orng_serve_submit(srv, out=b.data_ptr() + 4, **q))
        for q, t, b in zip(reqs, tickets, bufs):
            res = R.orng_serve_wait(srv, t)
            torch.cuda.synchronize()
            host = b.cpu().numpy().view(np.uint32)
            ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
            assert np.array_equal(host[1:1 + q["n"]], ref.view(np.uint32))
            assert host[0] == 0xFFFFFFFF and host[-1] == 0xFFFFFFFF
            R.orng_serve_release(srv, t)
        assert R.orng_serve_stats(srv)["steps"] >= 5  # requests spread over several steps
    finally:
        R.orng_serve_destroy(srv)


def test_serve_mix_equals_alone(R):
    rng = np.random.default_rng(3)
    probe = dict(gen=2, dist=2, seed=123456789, ctr=77, offset=1001, n=50_001)
    arena = _arena(32 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        t = R.orng_serve_submit(srv, **probe)
        alone = _read(arena, R.orng_serve_wait(srv, t)).copy()
        R.orng_serve_release(srv, t)
        others = _random_reqs(rng, 40)
        ts = [R.orng_serve_submit(srv, **q) for q in others[:20]]
        t = R.orng_serve_submit(srv, **probe)
        ts += [R.orng_serve_submit(srv, **q) for q in others[20:]]
        mixed = _read(arena, R.orng_serve_wait(srv, t))
        assert np.array_equal(alone, mixed)
        for x in ts:
            R.orng_serve_wait(srv, x)
            R.orng_serve_release(srv, x)
        R.orng_serve_release(srv, t)
    finally:
        R.orng_serve_destroy(srv)


def test_serve_admission_under_budget(R, O):
    """A 1 MiB arena holds one 200k-word output at a time: the next request is
    admitted only after the previous one is released."""
    arena = _arena(1 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        qs = [dict(gen=0, dist=0, seed=i, ctr=i, offset=0, n=200_000) for i in range(4)]
        ts = [R.orng_serve_submit(srv, **q) for q in qs]
        first = R.orng_serve_wait(srv, ts[0])
        time.sleep(0.05)
        assert R.orng_serve_poll(srv, ts[1]) is None  # still waiting for arena space
        st = R.orng_serve_stats(srv)
        assert st["admitted"] == 1 and st["queued"] == 3
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_release(srv, ts[1])
        assert e.value.status == R.EBUSY
        assert np.array_equal(_read(arena, first), O.fill(0, 0, 0, 0, 0, 200_000))
        R.orng_serve_release(srv, ts[0])
        for i in range(1, 4):
            res = R.orng_serve_wait(srv, ts[i])
            assert np.array_equal(_read(arena, res), O.fill(0, 0, i, i, 0, 200_000))
            R.orng_serve_release(srv, ts[i])
        assert R.orng_serve_stats(srv)["arena_peak_bytes"] <= 1 << 20
    finally:
        R.orng_serve_destroy(srv)


def test_serve_errors(R):
    arena = _arena(1 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit(srv, 0, 0, 1, 1, 0, 1 << 20)  # 4 MiB > 1 MiB arena
        assert e.value.status == R.ENOMEM
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit(srv, 10, 0, 1, 1, 0, 16)
        assert e.value.status == R.EINVAL
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit(srv, 9, 0, 2**32, 1, 0, 16)
        assert e.value.status == R.EINVAL
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit(srv, 0, 0, 1, 1, 2**32 - 4, 16)
        assert e.value.status == R.ERANGE
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_release(srv, 12345)
        assert e.value.status == R.ENOENT
        t = R.orng_serve_submit(srv, 0, 0, 1, 1, 0, 16)
        R.orng_serve_wait(srv, t)
        R.orng_serve_release(srv, t)
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_poll(srv, t)
        assert e.value.status == R.ENOENT
    finally:
        R.orng_serve_destroy(srv)


def test_serve_destroy_drains_in_flight(R, O):
    out = torch.full((1 << 20,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the server's streams do not wait for torch's
    srv = R.orng_serve_create(1 << 24)
    for k in range(8):
        R.orng_serve_submit(srv, 4, 1, k, k, 0, 1 << 17, out=out.data_ptr() + k * (1 << 19))
    R.orng_serve_destroy(srv)  # returns only after all queued work ran
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint32)
    for k in range(8):
        ref = O.fill(4, 1, k, k, 0, 1 << 17).view(np.uint32)
        assert np.array_equal(host[k * (1 << 17):(k + 1) * (1 << 17)], ref)


def test_serve_submit_many_and_release_many(R, O):
    rng = np.random.default_rng(7)
    qs = _random_reqs(rng, 50)
    arena = _arena(16 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        reqs = R.make_requests([q["gen"] for q in qs], [q["dist"] for q in qs],
                               [q["seed"] for q in qs], [q["ctr"] for q in qs],
                               [q["offset"] for q in qs], [q["n"] for q in qs], 0)
        tickets = R.orng_serve_submit_many(srv, reqs)
        assert len(set(tickets.tolist())) == 50
        for q, t in zip(qs[:10], tickets[:10]):
            res = R.orng_serve_wait(srv, int(t))
            ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
            assert np.array_equal(_read(arena, res), ref.view(np.uint32))
        assert R.orng_serve_release_many(srv, tickets) == 50
        st = R.orng_serve_stats(srv)
        assert st["released"] == 50 and st["completed"] == 50
        bad = R.make_requests([0, 10], 0, 1, 1, 0, 16, 0)
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit_many(srv, bad)
        assert e.value.status == R.EINVAL
        assert R.orng_serve_stats(srv)["submitted"] == 50  # nothing of the bad batch queued
    finally:
        R.orng_serve_destroy(srv)


def test_serve_trace_requests_sampled(R, O):
    """The first 400 requests of the serving workload (Poisson arrivals,
    sizes log-uniform in [2^10, 2^26] words, all generator families and
    distributions), submitted at once into a 16 GiB arena and checked on
    sampled positions (first, last and random words) against the oracle."""
    from paper_2310_19925_amd import inputs
    tr = inputs.serve_trace()
    m = 400
    assert int(tr["n"][:m].sum()) * 4 < (16 << 30)
    arena = _arena(16 << 30)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    rng = np.random.default_rng(9)
    try:
        reqs = R.make_requests(tr["gen"][:m], tr["dist"][:m], tr["seed"][:m], tr["ctr"][:m],
                               tr["offset"][:m], tr["n"][:m], 0)
        tickets = R.orng_serve_submit_many(srv, reqs)
        for i, t in enumerate(tickets):
            res = R.orng_serve_wait(srv, int(t))
            n = int(tr["n"][i])
            js = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 6)]))
            off = (res["d_out"] - arena.data_ptr()) // 4
            got = arena[torch.from_numpy(off + js).cuda()].cpu().numpy().view(np.uint32)
            ref = O.samples_at(int(tr["gen"][i]), int(tr["dist"][i]), int(tr["seed"][i]),
                               np.full(js.size, tr["ctr"][i], np.uint32),
                               (int(tr["offset"][i]) + js).astype(np.uint64))
            assert np.array_equal(got, ref.view(np.uint32)), ("request", i)
        assert R.orng_serve_release_many(srv, tickets) == m
    finally:
        R.orng_serve_destroy(srv)
    del arena
    torch.cuda.empty_cache()


def test_serve_destroy_with_unreleased_results_still_drains(R):
    """Finished results that the client never released fill the arena; destroy
    still runs the queued requests (their outputs die with the server)."""
    arena = _arena(1 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    ts = [R.orng_serve_submit(srv, 0, 0, i, i, 0, 200_000) for i in range(3)]
    assert R.orng_serve_wait(srv, ts[0]) is not None
    t0 = time.time()
    R.orng_serve_destroy(srv)  # must not wait for a release that never comes
    assert time.time() - t0 < 60


def test_serve_try_submit_admits_at_once_or_returns_eagain(R, O):
    """The non-blocking submit queues a request only when it can be admitted
    at once; otherwise it returns EAGAIN and queues nothing."""
    arena = _arena(1 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    try:
        big = dict(gen=0, dist=1, seed=5, ctr=6, offset=7, n=200_000)      # 800 KB
        t1 = R.orng_serve_try_submit(srv, **big)
        assert t1 is not None
        # the arena holds t1's range until it is released
        assert R.orng_serve_try_submit(srv, 3, 0, 1, 2, 3, 100_000) is None
        res = R.orng_serve_wait(srv, t1)
        assert np.array_equal(_read(arena, res), O.fill(0, 1, 5, 6, 7, 200_000).view(np.uint32))
        # a blocking submit that does not fit waits in the queue; a small
        # non-blocking one behind it is refused even though it would fit
        t2 = R.orng_serve_submit(srv, 4, 2, 8, 9, 10, 150_000)              # 600 KB
        time.sleep(0.05)
        assert R.orng_serve_poll(srv, t2) is None
        assert R.orng_serve_try_submit(srv, 0, 0, 1, 1, 0, 256) is None
        st = R.orng_serve_stats(srv)
        assert st["submitted"] == 2 and st["queued"] == 1
        R.orng_serve_release(srv, t1)
        res = R.orng_serve_wait(srv, t2)
        assert np.array_equal(_read(arena, res), O.fill(4, 2, 8, 9, 10, 150_000).view(np.uint32))
        t3 = R.orng_serve_try_submit(srv, 0, 0, 1, 1, 0, 256)
        assert t3 is not None
        res = R.orng_serve_wait(srv, t3)
        assert np.array_equal(_read(arena, res), O.fill(0, 0, 1, 1, 0, 256).view(np.uint32))
        R.orng_serve_release(srv, t2)
        R.orng_serve_release(srv, t3)
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_try_submit(srv, 0, 0, 1, 1, 0, 1 << 20)  # larger than the arena
        assert e.value.status == R.ENOMEM
    finally:
        R.orng_serve_destroy(srv)


def _failing_server(R, monkeypatch, step, **kw):
    """A server whose step number `step` fails on the host before anything of
    it is enqueued (the environment hook is read when the server is made)."""
    monkeypatch.setenv("ORNG_SERVE_FAIL_STEP", str(step))
    try:
        return R.orng_serve_create(**kw)
    finally:
        monkeypatch.delenv("ORNG_SERVE_FAIL_STEP")


def test_serve_first_step_failure_fails_every_ticket(R, monkeypatch):
    print("serve: injected failure of step 1", flush=True)
    arena = _arena(16 << 20)
    srv = _failing_server(R, monkeypatch, 1, arena_bytes=arena.numel() * 4, arena=arena)
    rng = np.random.default_rng(21)
    qs = _random_reqs(rng, 12, 10, 14)
    reqs = R.make_requests([q["gen"] for q in qs], [q["dist"] for q in qs],
                           [q["seed"] for q in qs], [q["ctr"] for q in qs],
                           [q["offset"] for q in qs], [q["n"] for q in qs], 0)
    tickets = R.orng_serve_submit_many(srv, reqs)
    for t in tickets:
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_wait(srv, int(t), timeout_ns=30_000_000_000)
        assert e.value.status == R.EHIP
    with pytest.raises(R.OrngError) as e:
        R.orng_serve_submit(srv, 0, 0, 1, 1, 0, 16)
    assert e.value.status == R.EHIP
    st = R.orng_serve_stats(srv)
    assert st["failed"] == 12 and st["completed"] == 0
    t0 = time.time()
    with pytest.raises(R.OrngError) as e:
        R.orng_serve_destroy(srv)
    assert e.value.status == R.EHIP and time.time() - t0 < 30


def test_serve_later_step_failure_keeps_finished_results(R, O, monkeypatch):
    """Step 3 fails: the two steps queued before it are waited for, requests
    they finished end done with the right words, every other ticket ends
    EHIP, and nothing is left running."""
    print("serve: injected failure of step 3", flush=True)
    outs = torch.full((40, 1 << 14), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the server's streams do not wait for torch's
    srv = _failing_server(R, monkeypatch, 3, arena_bytes=1 << 20, step_words=1 << 15)
    qs = [dict(gen=k % 9, dist=k % 3, seed=1000 + k, ctr=k, offset=3 * k, n=(1 << 14) - k)
          for k in range(40)]
    reqs = R.make_requests([q["gen"] for q in qs], [q["dist"] for q in qs],
                           [q["seed"] for q in qs], [q["ctr"] for q in qs],
                           [q["offset"] for q in qs], [q["n"] for q in qs],
                           outs.data_ptr() + outs.stride(0) * 4 * np.arange(40))
    tickets = R.orng_serve_submit_many(srv, reqs)
    done, failed = [], []
    for k, t in enumerate(tickets):
        try:
            res = R.orng_serve_wait(srv, int(t), timeout_ns=30_000_000_000)
            assert res is not None, "ticket still running after the failure"
            done.append(k)
        except R.OrngError as e:
            assert e.status == R.EHIP
            failed.append(k)
    assert failed, "the injected failure failed no request"
    host = outs.cpu().numpy().view(np.uint32)
    for k in done:
        q = qs[k]
        ref = O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"])
        assert np.array_equal(host[k, :q["n"]], ref.view(np.uint32)), ("request", k)
    st = R.orng_serve_stats(srv)
    assert st["failed"] == len(failed) and st["completed"] == len(done)
    assert st["steps"] == 2
    with pytest.raises(R.OrngError) as e:
        R.orng_serve_destroy(srv)
    assert e.value.status == R.EHIP


def test_serve_saturated_trace_every_result(R, O):
    """The whole serving workload (20,000 requests: sizes log-uniform in
    [2^10, 2^26] words, every generator family and distribution) submitted at
    once into a 32 GB arena, as in the saturated replay: every served output
    equals orng_fill of the same request in full (compared on the device), and
    its first, last and four random samples equal the oracle's."""
    from paper_2310_19925_amd import inputs
    tr = inputs.serve_trace()
    m = tr["n"].size
    arena = _arena(32_000_000_000 // 256 * 256)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena)
    ref = torch.empty(int(tr["n"].max()), dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(13)
    gathered, wanted = [], []
    print("serve: saturated trace of %d requests" % m, flush=True)
    try:
        reqs = R.make_requests(tr["gen"], tr["dist"], tr["seed"], tr["ctr"], tr["offset"],
                               tr["n"], 0)
        tickets = R.orng_serve_submit_many(srv, reqs)
        for i, t in enumerate(tickets):
            res = R.orng_serve_wait(srv, int(t))
            n = int(tr["n"][i])
            g, d = int(tr["gen"][i]), int(tr["dist"][i])
            out = ref[:n]
            R.orng_fill(g, d, int(tr["seed"][i]), int(tr["ctr"][i]), int(tr["offset"][i]), n, out)
            off = (res["d_out"] - arena.data_ptr()) // 4
            view = arena[off:off + n]
            assert torch.equal(view, out), ("request", i)
            js = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 4)]))
            gathered.append(view[torch.from_numpy(js).cuda()])
            wanted.append((g, d, i, js))
            R.orng_serve_release(srv, int(t))
            if (i + 1) % 5000 == 0:
                print("serve: %d results checked" % (i + 1), flush=True)
        st = R.orng_serve_stats(srv)
        assert st["completed"] == m and st["failed"] == 0
    finally:
        R.orng_serve_destroy(srv)
    got = torch.cat(gathered).cpu().numpy().view(np.uint32)
    del arena, ref
    torch.cuda.empty_cache()
    k = 0
    for g, d, i, js in wanted:
        exp = O.samples_at(g, d, int(tr["seed"][i]), np.full(js.size, tr["ctr"][i], np.uint32),
                           (int(tr["offset"][i]) + js).astype(np.uint64))
        assert np.array_equal(got[k:k + js.size], exp.view(np.uint32)), ("request", i)
        k += js.size


def _range_reqs(rng, m, lo_log2=10, hi_log2=16):
    """Integer-range requests: every generator, bounds from one value to the
    whole int32 span, offsets anywhere in the 2^31 samples of a stream."""
    out = []
    for k in range(m):
        n = int(2 ** (lo_log2 + (hi_log2 - lo_log2) * rng.random()))
        lo = int(rng.integers(-2**31, 2**31 - 1))
        r = [2**32 - 1, 1, 6, int(2 ** rng.integers(1, 32)), int(rng.integers(1, 2**32))][k % 5]
        lo = -2**31 if r == 2**32 - 1 else lo
        hi = min(lo + r, 2**31 - 1)
        q = dict(gen=int(rng.integers(0, 10)), dist=5, seed=int(rng.integers(0, 2**63)),
                 ctr=int(rng.integers(0, 2**32)), offset=int(rng.integers(0, 2**31 - n)), n=n,
                 lo=lo, hi=hi)
        if q["gen"] == 9:
            q["seed"] &= 0xFFFFFFFF
        out.append(q)
    return out


def _ref(O, q):
    if q["dist"] == 5:
        return O.fill_range(q["gen"], q["seed"], q["ctr"], 1, q["offset"], q["n"], q["lo"],
                            q["hi"]).view(np.uint32)
    return O.fill(q["gen"], q["dist"], q["seed"], q["ctr"], q["offset"], q["n"]).view(np.uint32)


def test_serve_integer_ranges(R, O):
    """Integer-range requests served in a mix with other distributions, into
    arena outputs and misaligned caller buffers, several steps per request:
    each equals orng_fill_range of the same stream and bounds (the oracle's)
    and the same request served alone."""
    rng = np.random.default_rng(21)
    f64 = [dict(q, dist=4 if k % 2 else 3, offset=max(0, q["offset"] // 2 - q["n"]))
           for k, q in enumerate(_random_reqs(rng, 10))]  # float64 in the same steps
    qs = _range_reqs(rng, 40) + _random_reqs(rng, 40) + f64
    qs = [qs[i] for i in rng.permutation(len(qs))]
    arena = _arena(32 << 20)
    srv = R.orng_serve_create(arena.numel() * 4, arena=arena, step_words=1 << 16)
    try:
        bufs, tickets = [], []
        for k, q in enumerate(qs):
            w = 2 * q["n"] if q["dist"] in (3, 4) else q["n"]  # output words
            if k % 3 == 0:  # caller buffer, one word off the 16-byte grid (two for float64)
                sh = 2 if q["dist"] in (3, 4) else 1
                b = torch.full((w + sh + 1,), -1, dtype=torch.int32, device="cuda")
                torch.cuda.synchronize()  # the server's streams do not wait for torch's
                bufs.append((b, sh, w))
                tickets.append(R.orng_serve_submit(srv, out=b.data_ptr() + 4 * sh, **q))
            else:
                bufs.append(None)
                tickets.append(R.orng_serve_submit(srv, **q))
        for q, t, b in zip(qs, tickets, bufs):
            res = R.orng_serve_wait(srv, t)
            assert res["status"] == 0 and res["n"] == q["n"]
            if b is None:
                w = 2 * q["n"] if q["dist"] in (3, 4) else q["n"]
                off = (res["d_out"] - arena.data_ptr()) // 4
                torch.cuda.synchronize()
                got = arena[off:off + w].cpu().numpy().view(np.uint32)
            else:
                buf, sh, w = b
                torch.cuda.synchronize()
                host = buf.cpu().numpy().view(np.uint32)
                assert np.all(host[:sh] == 0xFFFFFFFF) and host[-1] == 0xFFFFFFFF
                got = host[sh:sh + w]
            assert np.array_equal(got, _ref(O, q)), q
            R.orng_serve_release(srv, t)
        # mix == alone for one range request
        probe = _range_reqs(rng, 1, 16, 17)[0]
        t = R.orng_serve_submit(srv, **probe)
        alone = _read(arena, R.orng_serve_wait(srv, t)).copy()
        R.orng_serve_release(srv, t)
        others = _random_reqs(rng, 20) + _range_reqs(rng, 20)
        ts = [R.orng_serve_submit(srv, **q) for q in others[:20]]
        t = R.orng_serve_submit(srv, **probe)
        ts += [R.orng_serve_submit(srv, **q) for q in others[20:]]
        assert np.array_equal(_read(arena, R.orng_serve_wait(srv, t)), alone)
        R.orng_serve_release(srv, t)
        for x in ts:
            R.orng_serve_wait(srv, x)
            R.orng_serve_release(srv, x)
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit(srv, 0, 5, 1, 1, 0, 16, lo=3, hi=3)
        assert e.value.status == R.EINVAL
        with pytest.raises(R.OrngError) as e:
            R.orng_serve_submit(srv, 0, 5, 1, 1, 2**31 - 4, 16, lo=0, hi=3)
        assert e.value.status == R.ERANGE
    finally:
        R.orng_serve_destroy(srv)
