"""Pins for the oracle environment: hand-worked steps, invariants, edge cases.

The hand-worked steps follow the MDP of Section 3.1 and the step / reward
operations of Section 4.2; the invariants are consequences of those
definitions (conservation of cash plus holdings net of costs, rewards that
telescope to the change in total assets, zero orders leaving the account
untouched).
"""
import json
import os

import numpy as np
import pytest

from oracle.env import OracleEnv, buy_quantity, execute_trades, orders, portfolio_value
from workload import EnvConfig, make_actions, make_market

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked_steps.json")


def _fx(s):
    return float.fromhex(s)


def _one_step(case, cost_rate, hmax):
    """Run one oracle step on a 2-stock, 1-env market built from a fixture case."""
    p_t = np.array(case["p_t"], dtype=np.float32)
    p_t1 = np.array(case["p_t1"], dtype=np.float32)
    close = np.stack([p_t, p_t1])
    ind = np.zeros((2, 1, 2), dtype=np.float32)
    cfg = EnvConfig(n_envs=1, n_stocks=2, n_ind=1, n_days=1, hmax=hmax, cost_rate=cost_rate,
                    init_cash=_fx(case["cash"]), reward_scale=_fx(case["reward_scale"]))
    env = OracleEnv(cfg, close, ind)
    env.hold[:] = np.array(case["hold"], dtype=np.int32)
    env.asset = portfolio_value(env.cash, env.hold, close[0])
    a = np.array([case["action"]], dtype=np.float32)
    q = orders(a, hmax)
    v_t = env.asset.copy()
    _, r, x, done = env.step(a)
    return dict(q=q[0], x=x[0], hold=env.hold[0], cash=env.cash[0], v_t=v_t[0], v_t1=env.asset[0], r=r[0],
                done=done)


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_hand_worked_steps(golden):
    for case in golden["cases"]:
        out = _one_step(case, golden["cost_rate"], golden["hmax"])
        assert list(out["q"]) == case["expect_orders"], case["name"]
        assert list(out["x"]) == case["expect_exec"], case["name"]
        assert list(out["hold"]) == case["expect_hold"], case["name"]
        if "expect_cash" in case:
            assert out["cash"] == _fx(case["expect_cash"]), (case["name"], out["cash"].hex())
        if "expect_v_t" in case:
            assert out["v_t"] == _fx(case["expect_v_t"]), case["name"]
            assert out["v_t1"] == _fx(case["expect_v_t1"]), case["name"]
        if "expect_reward" in case:
            assert out["r"] == _fx(case["expect_reward"]), (case["name"], float(out["r"]).hex())
        assert out["done"]


def test_truncation_uses_float32_product(golden):
    tr = golden["truncation"]
    a = np.array(tr["action"], dtype=np.float32)
    assert list(orders(a, golden["hmax"])) == tr["expect_orders"]
    # The float64 product of the same inputs gives different orders: the float32 rounding is normative.
    f64 = np.trunc(a.astype(np.float64) * 100.0).astype(int)
    assert list(f64) == tr["float64_product_orders"]


def test_orders_clamp_and_nan():
    a = np.array([np.nan, 3.0, -7.5, np.inf, -np.inf, 1.0000001], dtype=np.float32)
    assert list(orders(a, 100)) == [0, 100, -100, 100, -100, 100]


def test_buy_boundary_is_inclusive():
    one_p = 1.0 + 1e-3
    cost3 = (100.0 * 3.0) * one_p
    k = buy_quantity(np.array([cost3, np.nextafter(cost3, 0.0), 0.0, 1e9]), 100.0, np.array([5, 5, 5, 5]), one_p)
    assert list(k) == [3, 2, 0, 5]


def test_buy_quantity_matches_linear_scan():
    rng = np.random.default_rng(3)
    one_p = 1.0 + 1e-3
    for _ in range(20):
        price = float(np.float32(rng.uniform(1, 400)))
        cash = rng.uniform(0, 5000, size=200)
        q = rng.integers(0, 101, size=200)
        k = buy_quantity(cash, price, q, one_p)
        for i in range(200):
            best = 0
            for kk in range(int(q[i]) + 1):
                if (price * kk) * one_p <= cash[i]:
                    best = kk
            assert k[i] == best


def _run(seed, n_envs=48, n_days=30, n_stocks=30, buy_bias=0.15, scale=1.0):
    m = make_market(seed, n_stocks, n_days)
    cfg = EnvConfig(n_envs=n_envs, n_stocks=n_stocks, n_days=n_days)
    env = OracleEnv(cfg, m.close, m.ind)
    env.reset()
    acts = make_actions(seed + 1, n_days, n_envs, n_stocks, buy_bias=buy_bias) * np.float32(scale)
    return m, cfg, env, acts


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_conservation_and_bounds(seed):
    """After trading at p_t: cash' + p_t.h' = cash + p_t.h - c * sum_d p_t,d |x_d| (up to rounding)."""
    m, cfg, env, acts = _run(seed)
    for t in range(cfg.n_days):
        p = m.close[t].astype(np.float64)
        cash0, h0 = env.cash.copy(), env.hold.copy()
        _, _, x, _ = env.step(acts[t])
        lhs = env.cash + env.hold.astype(np.float64) @ p
        rhs = cash0 + h0.astype(np.float64) @ p - cfg.cost_rate * (np.abs(x).astype(np.float64) @ p)
        scale = np.maximum(np.abs(cash0 + h0 @ p), 1.0)
        assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale)
        assert np.all(env.hold >= 0)
        assert np.all(env.cash >= 0)
        assert np.all(np.abs(x) <= cfg.hmax)
        assert np.array_equal(env.hold, h0 + x)


@pytest.mark.parametrize("seed", [21, 22])
def test_rewards_telescope(seed):
    """R_T = (v_T - v_0) * scale and v_T - v_0 = sum_t [(p_t+1 - p_t).h_t+1 - c p_t.|x_t|]."""
    m, cfg, env, acts = _run(seed)
    v0 = env.asset.copy()
    decomposed = np.zeros(cfg.n_envs)
    for t in range(cfg.n_days):
        _, _, x, _ = env.step(acts[t])
        dp = m.close[t + 1].astype(np.float64) - m.close[t].astype(np.float64)
        decomposed += env.hold.astype(np.float64) @ dp - cfg.cost_rate * (np.abs(x) @ m.close[t].astype(np.float64))
    tol = 1e-12 * np.maximum(np.abs(v0), np.abs(env.asset))
    assert np.all(np.abs(env.cumrew / cfg.reward_scale - (env.asset - v0)) <= tol * cfg.n_days)
    assert np.all(np.abs(decomposed - (env.asset - v0)) <= tol * cfg.n_days)


def test_zero_action_invariant():
    """Every |a| < 0.01 gives zero orders: cash and holdings unchanged, assets move with prices only."""
    m, cfg, env, acts = _run(31, buy_bias=0.3)
    for t in range(10):                         # build positions first
        env.step(acts[t])
    rng = np.random.default_rng(5)
    for t in range(10, cfg.n_days):
        a = rng.uniform(-0.0099, 0.0099, size=(cfg.n_envs, cfg.n_stocks)).astype(np.float32)
        cash0, h0, v0 = env.cash.copy(), env.hold.copy(), env.asset.copy()
        _, r, x, _ = env.step(a)
        assert np.array_equal(env.cash, cash0)
        assert np.array_equal(env.hold, h0)
        assert not x.any()
        dp = m.close[t + 1].astype(np.float64) - m.close[t].astype(np.float64)
        assert np.all(np.abs(r / cfg.reward_scale - h0 @ dp) <= 1e-12 * np.abs(v0))


def test_sells_cannot_short_and_buys_cannot_overdraw():
    m, cfg, env, _ = _run(41, n_envs=8, n_days=5)
    env.step(np.full((8, 30), -1.0, np.float32))            # sell with nothing held
    assert not env.hold.any() and np.all(env.cash == cfg.init_cash)
    for _ in range(4):
        env.step(np.full((8, 30), 1.0, np.float32))         # buy 100 of everything until cash binds
        assert np.all(env.cash >= 0)
    assert np.all(env.cash < np.min(m.close[3:5]) * 1.001 * 100 * 30)


def test_state_roundtrip_resumes_bit_identically():
    m, cfg, env, acts = _run(51, n_envs=16)
    for t in range(12):
        env.step(acts[t])
    snap = env.get_state()
    tail_a = [env.step(acts[t]) for t in range(12, cfg.n_days)]
    env2 = OracleEnv(cfg, m.close, m.ind)
    env2.set_state(snap)
    tail_b = [env2.step(acts[t]) for t in range(12, cfg.n_days)]
    for (oa, ra, xa, _), (ob, rb, xb, _) in zip(tail_a, tail_b):
        assert np.array_equal(oa, ob) and np.array_equal(ra, rb) and np.array_equal(xa, xb)


def test_step_past_horizon_raises():
    m, cfg, env, acts = _run(61, n_envs=2, n_days=3)
    for t in range(3):
        env.step(acts[t])
    with pytest.raises(RuntimeError):
        env.step(acts[0])


def test_obs_layout_and_scaling():
    m, cfg, env, acts = _run(71, n_envs=4, n_days=4)
    env.step(acts[0])
    o = env.obs()
    D, I = cfg.n_stocks, cfg.n_ind
    assert o.shape == (4, (I + 2) * D + 1) and o.dtype == np.float32
    assert np.array_equal(o[:, 0], (env.cash * 2.0 ** -20).astype(np.float32))
    assert np.array_equal(o[:, 1:1 + D], np.broadcast_to(m.close[1] / 256.0, (4, D)))
    assert np.array_equal(o[:, 1 + D:1 + 2 * D], env.hold.astype(np.float32) / 1024.0)
    assert np.array_equal(o[:, 1 + 2 * D:], np.broadcast_to(m.ind[1].reshape(-1), (4, I * D)))
