"""GPU parity of the fused Brownian walk against the oracle (bit-exact
positions) and its mean squared displacement against 2 * dim * D * t."""
import math

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


def _walk(R, seed, ctr0, n, dim, step0, steps, dt, D, pos=None, msd_every=0):
    p = torch.zeros((dim, n), dtype=torch.float32, device="cuda") if pos is None else \
        torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    nsnap = steps // msd_every if msd_every else 0
    msd = torch.full((max(nsnap, 1),), -1.0, dtype=torch.float64, device="cuda")
    R.orng_brownian(seed, ctr0, n, dim, step0, steps, dt, D, p, msd if nsnap else None, msd_every)
    torch.cuda.synchronize()
    return p.cpu().numpy(), (msd.cpu().numpy()[:nsnap] if nsnap else None)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_walk_parity_small(R, O, dim):
    for n, step0, steps in [(1000, 0, 300), (777, 5, 101), (64, 1001, 3), (300, 0, 1)]:
        print("walk dim=%d n=%d step0=%d steps=%d" % (dim, n, step0, steps), flush=True)
        rng = np.random.default_rng(n)
        start = rng.standard_normal((dim, n)).astype(np.float32)
        got, msd = _walk(R, 2**40 + 3, 17, n, dim, step0, steps, 1e-3, 1.0, pos=start,
                         msd_every=max(1, steps // 3))
        ref, rmsd = O.brownian(2**40 + 3, 17, n_particles=n, dim=dim, step0=step0, n_steps=steps,
                               dt=1e-3, D=1.0, pos=start, msd_every=max(1, steps // 3))
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        assert np.allclose(msd, rmsd, rtol=1e-12, atol=0)


def test_walk_resume_and_zero(R):
    a, _ = _walk(R, 9, 0, 5000, 3, 0, 200, 1e-3, 1.0)
    h, _ = _walk(R, 9, 0, 5000, 3, 0, 100, 1e-3, 1.0)
    b, _ = _walk(R, 9, 0, 5000, 3, 100, 100, 1e-3, 1.0, pos=h)
    assert np.array_equal(a, b)
    z, m = _walk(R, 9, 0, 5000, 3, 0, 50, 1e-3, 0.0, msd_every=10)
    assert not z.any() and not m.any()


def test_walk_errors(R):
    p = torch.zeros((3, 4), dtype=torch.float32, device="cuda")
    for args in [(1, 0, 4, 4, 0, 1, 1e-3, 1.0), (1, 0, 4, 0, 0, 1, 1e-3, 1.0),
                 (1, 0, 4, 3, 0, 1, 1e-3, -1.0)]:
        with pytest.raises(R.OrngError) as e:
            R.orng_brownian(*args, p)
        assert e.value.status == R.EINVAL
    with pytest.raises(R.OrngError) as e:
        R.orng_brownian(1, 0, 4, 3, 2**32 // 3, 2, 1e-3, 1.0, p)
    assert e.value.status == R.ERANGE
    with pytest.raises(R.OrngError) as e:
        R.orng_brownian(1, 2**32 - 2, 4, 3, 0, 2, 1e-3, 1.0, p)
    assert e.value.status == R.ERANGE


def test_walk_full_config(R, O):
    """2^24 particles, 3-D, 10^4 steps, dt = 1e-3, D = 1, from the origin, in
    one launch: a seeded subset of 65,536 particles spread over all ids (plus
    the first and last) bit-exact against the oracle over all 10^4 steps, and
    the MSD of all particles against 6 t."""
    from paper_2310_19925_amd import inputs
    cfg = inputs.WALK
    n, dim, steps = cfg["n_particles"], cfg["dim"], cfg["n_steps"]
    seed = inputs.bulk_seed()
    pos = torch.zeros((dim, n), dtype=torch.float32, device="cuda")
    msd = torch.zeros(steps // cfg["msd_every"], dtype=torch.float64, device="cuda")
    R.orng_brownian(seed, 0, n, dim, 0, steps, cfg["dt"], cfg["D"], pos, msd, cfg["msd_every"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    ids = np.unique(np.concatenate([rng.choice(n, 65536, replace=False), [0, 1, n - 1]]))
    ids = ids.astype(np.uint32)
    got = pos[:, torch.from_numpy(ids.astype(np.int64)).cuda()].cpu().numpy()
    print("walk: oracle on %d particles x %d steps" % (ids.size, steps), flush=True)
    ref, _ = O.brownian(seed, 0, ids=ids, dim=dim, n_steps=steps, dt=cfg["dt"], D=cfg["D"])
    bad = np.nonzero((got.view(np.uint32) != ref.view(np.uint32)).any(axis=0))[0]
    assert bad.size == 0, "%d particles differ, first id %d" % (bad.size, ids[bad[0]])
    m = msd.cpu().numpy() / n
    for q, val in enumerate(m):
        t = (q + 1) * cfg["msd_every"] * cfg["dt"]
        expect = 2 * dim * cfg["D"] * t
        se = 2 * cfg["D"] * t * math.sqrt(2 * dim) / math.sqrt(n)
        assert abs(val - expect) < 5 * se, (t, val, expect)
    # the last snapshot is the MSD of the final positions
    final = float((pos.double() ** 2).sum()) / n
    assert math.isclose(final, m[-1], rel_tol=1e-9)


def test_walk_all_particles_100_steps(R, O):
    """All 2^24 particles of the configured walk for 100 steps (a separate
    launch in the benchmark's launch configuration), every position bit-exact
    against the oracle."""
    from paper_2310_19925_amd import inputs
    cfg = inputs.WALK
    n, dim, seed = cfg["n_particles"], cfg["dim"], inputs.bulk_seed()
    print("walk all %d particles x 100 steps" % n, flush=True)
    pos = torch.zeros((dim, n), dtype=torch.float32, device="cuda")
    R.orng_brownian(seed, 0, n, dim, 0, 100, cfg["dt"], cfg["D"], pos)
    torch.cuda.synchronize()
    got = pos.cpu().numpy()
    ref, _ = O.brownian(seed, 0, n_particles=n, dim=dim, n_steps=100, dt=cfg["dt"], D=cfg["D"])
    bad = np.nonzero((got.view(np.uint32) != ref.view(np.uint32)).any(axis=0))[0]
    assert bad.size == 0, "%d particles differ, first %d" % (bad.size, bad[0])


def test_walk_largest_particle_count(R, O):
    """2^32 - 1 particles (1-D, 16 GiB of positions), two steps: the grid
    covers every particle (its workgroup count is rounded up without
    wrapping); the first and last 1,000 particles against the oracle, whose
    particle i0 + j of a walk with counter base 0 is particle j of one with
    counter base i0."""
    n = 2**32 - 1
    print("walk n=%d dim=1 steps=2" % n, flush=True)
    pos = torch.zeros((1, n), dtype=torch.float32, device="cuda")
    R.orng_brownian(77, 0, n, 1, 0, 2, 1e-3, 1.0, pos, None, 0)
    torch.cuda.synchronize()
    for i0 in (0, n - 1000):
        got = pos[0, i0:i0 + 1000].cpu().numpy()
        ref, _ = O.brownian(77, i0, n_particles=1000, dim=1, n_steps=2, dt=1e-3, D=1.0)
        assert np.array_equal(got.view(np.uint32), ref.ravel().view(np.uint32)), i0
    del pos
    torch.cuda.empty_cache()
