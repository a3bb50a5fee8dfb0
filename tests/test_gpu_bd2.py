"""GPU parity of the paper's 2-D Brownian dynamics example (orng_bd2) with
the oracle, bit for bit on all four float64 state arrays, for one launch per
step, several steps per launch and all steps in one launch."""
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


def _state(n, rng=None):
    if rng is None:
        return np.zeros((4, n), np.float64)
    return rng.standard_normal((4, n)) * np.array([[1.0], [1.0], [0.3], [0.3]])


def _run(R, st, pid0, step0, n_steps, dt, c, spl):
    d = torch.from_numpy(np.ascontiguousarray(st)).cuda()
    R.orng_bd2(pid0, st.shape[1], step0, n_steps, dt, c, d[0], d[1], d[2], d[3], spl)
    torch.cuda.synchronize()
    return d.cpu().numpy()


@pytest.mark.parametrize("spl", [0, 1, 5])
def test_bd2_parity_small(R, O, spl):
    rng = np.random.default_rng(5)
    n, pid0, step0, T, dt, c = 1000, 123, 5, 37, 3e-3, 2.5
    st = _state(n, rng)
    got = _run(R, st, pid0, step0, T, dt, c, spl)
    ref = O.bd2(pid0, n, step0=step0, n_steps=T, dt=dt, c=c, state=st)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


def test_bd2_high_pid_and_ragged(R, O):
    rng = np.random.default_rng(6)
    n, pid0 = 300, (1 << 40) + 7
    st = _state(n, rng)
    got = _run(R, st, pid0, 2**32 - 20, 20, 1e-2, 0.7, 0)  # ends on the last counter
    ref = O.bd2(pid0, n, step0=2**32 - 20, n_steps=20, dt=1e-2, c=0.7, state=st)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


def test_bd2_resume_continues_the_run(R):
    n = 4097
    a = _run(R, _state(n), 9, 1, 30, 1e-3, 1.0, 0)
    b = _run(R, _run(R, _state(n), 9, 1, 12, 1e-3, 1.0, 0), 9, 13, 18, 1e-3, 1.0, 7)
    assert np.array_equal(a.view(np.int64), b.view(np.int64))


def test_bd2_one_launch_per_step_equals_fused(R):
    n, T = 1 << 17, 200
    st = _state(n, np.random.default_rng(8))
    a = _run(R, st, 0, 1, T, 1e-3, 1.0, 1)
    b = _run(R, st, 0, 1, T, 1e-3, 1.0, 0)
    assert np.array_equal(a.view(np.int64), b.view(np.int64))


def test_bd2_paper_config_sampled(R, O):
    """The paper's run (10^6 particles, 10^4 steps) in one launch: sampled
    particles bit-exact against the oracle, and the whole population's
    velocity variance against the stationary AR(1) value."""
    from paper_2310_19925_amd import inputs
    p = inputs.BD2
    n, T = p["n"], p["n_steps"]
    got = _run(R, _state(n), p["pid0"], p["step0"], T, p["dt"], p["gamma_over_m"], 0)
    rng = np.random.default_rng(10)
    ids = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 64)])).astype(np.uint32)
    ref = O.bd2(p["pid0"], ids=ids, step0=p["step0"], n_steps=T, dt=p["dt"],
                c=p["gamma_over_m"])
    assert np.array_equal(got[:, ids].view(np.int64), ref.view(np.int64))
    a = 1.0 - p["gamma_over_m"] * p["dt"]
    var_v = p["dt"] / 3.0 * (1 - a ** (2 * T)) / (1 - a * a)
    for comp in (2, 3):
        assert abs(got[comp].var() / var_v - 1) < 5 * np.sqrt(2.0 / n)
    assert abs(np.corrcoef(got[2], got[3])[0, 1]) < 5 / np.sqrt(n)
