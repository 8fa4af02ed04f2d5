"""Property tests of the oracles over random markets, actions and sizes (hypothesis): the
invariants that the MDP of Section 3.1 fixes for any input, for the stock and the crypto task."""
import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

from oracle import crypto as oc
from oracle.env import OracleEnv, orders
from oracle.philox import philox4x64_10, uniforms_from_words
from workload import EnvConfig

SETTINGS = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@st.composite
def stock_case(draw):
    D = draw(st.integers(1, 6))
    N = draw(st.integers(1, 5))
    T = draw(st.integers(1, 4))
    I = draw(st.integers(0, 2))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    close = rng.uniform(1.0, 500.0, size=(T + 1, D)).astype(np.float32)
    ind = rng.standard_normal((T + 1, I, D)).astype(np.float32)
    acts = rng.uniform(-1.5, 1.5, size=(T, N, D)).astype(np.float32)
    acts[rng.random(acts.shape) < 0.05] = np.nan
    cash = draw(st.sampled_from([0.0, 100.0, 5e3, 1e6]))
    cost = draw(st.sampled_from([0.0, 1e-3, 0.05]))
    return EnvConfig(n_envs=N, n_stocks=D, n_ind=I, n_days=T, init_cash=cash, cost_rate=cost), close, ind, acts


@SETTINGS
@given(stock_case())
def test_stock_step_invariants(case):
    cfg, close, ind, acts = case
    env = OracleEnv(cfg, close, ind)
    env.reset()
    v0 = env.asset.copy()
    for t in range(cfg.n_days):
        cash0, h0 = env.cash.copy(), env.hold.copy()
        q = orders(acts[t], cfg.hmax)
        _, r, x, _ = env.step(acts[t])
        p = close[t].astype(np.float64)
        # Bounds: no shorting, no overdraft, fills within the orders.
        assert (env.hold >= 0).all() and (env.cash >= 0).all()
        assert (np.abs(x) <= np.abs(q)).all() and (np.abs(q) <= cfg.hmax).all()
        assert ((x == 0) | (np.sign(x) == np.sign(q))).all()
        assert np.array_equal(env.hold, h0 + x)
        # Conservation at p_t net of the proportional cost.
        lhs = env.cash + env.hold.astype(np.float64) @ p
        rhs = cash0 + h0.astype(np.float64) @ p - cfg.cost_rate * (np.abs(x).astype(np.float64) @ p)
        assert np.all(np.abs(lhs - rhs) <= 1e-12 * np.maximum(np.abs(rhs), 1.0))
    tol = 1e-12 * np.maximum(np.maximum(np.abs(v0), np.abs(env.asset)), 1.0) * cfg.n_days
    assert np.all(np.abs(env.cumrew / cfg.reward_scale - (env.asset - v0)) <= tol)


@SETTINGS
@given(st.integers(1, 6), st.integers(1, 40), st.sampled_from([0.0, 2e-4, 1e-2]), st.integers(0, 2 ** 31 - 1))
def test_crypto_step_invariants(n, T, fee, seed):
    rng = np.random.default_rng(seed)
    mid = 1000.0 * np.exp(np.cumsum(rng.standard_normal(T + 1) * 1e-3))
    acts = rng.integers(0, 3, size=(T, n))
    st_ = oc.CryptoState(n, 1e5)
    total = np.zeros(n)
    fees = np.zeros(n)
    prev = np.zeros(n, dtype=np.int64)
    for t in range(T):
        total += oc.step(st_, acts[t], np.full(n, mid[t]), np.full(n, mid[t + 1]), fee)
        assert set(np.unique(st_.pos)) <= {-1, 0, 1}
        fees += np.abs(st_.pos - prev) * mid[t] * fee
        prev = st_.pos.copy()
        assert (st_.peak >= st_.value).all() and (st_.mdd >= 0).all() and (st_.mdd >= st_.peak - st_.value).all()
    pos = acts - 1
    pnl = (pos * (mid[1:, None] - mid[:-1, None])).sum(0)
    np.testing.assert_allclose(total, pnl - fees, rtol=0, atol=1e-6)
    np.testing.assert_allclose(st_.sum_r, total, rtol=0, atol=1e-9)


@SETTINGS
@given(st.lists(st.integers(0, 2 ** 64 - 1), min_size=4, max_size=4), st.integers(0, 2 ** 64 - 1))
def test_philox_uniforms_in_open_interval_and_exact_in_float32(ctr, key):
    w = philox4x64_10(np.array(ctr, dtype=np.uint64)[None, :], np.array([key, 0], dtype=np.uint64))
    u = uniforms_from_words(w)
    assert ((u > 0) & (u < 1)).all()
    assert (u.astype(np.float32).astype(np.float64) == u).all()
