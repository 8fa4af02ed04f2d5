"""Oracle trading environment (TEST INFRASTRUCTURE ONLY; see the package docstring).

Follows the MDP of Section 3.1 and the reset / step / reward operations of
Section 4.2.  Readings of points the paper leaves open:

  * Orders: an action a in [-1, 1] asks for q = trunc(fl32(a * hmax)) shares
    (the product is rounded in float32, then truncated toward zero).  The
    action is clamped to [-1, 1] first and NaN counts as 0.  a > 0 buys,
    a < 0 sells, 0 holds (Section 3.1, Action).
  * No short positions (h_t is non-negative in Section 3.1): a sell is capped
    at the current holding.
  * All sells execute first in ascending stock order, then all buys in
    ascending stock order, at the day-t close p_t (the price in the state the
    action was chosen on).  Cash is float64 and every operation rounds once.
  * Proportional transaction cost c (Section 3.2 lists transaction costs among
    the market constraints): a sale of s shares credits (p*s)*(1-c); a buy of
    k shares debits (p*k)*(1+c), with 1-c and 1+c rounded to float64 once.
  * A buy fills the largest k in [0, q] whose debit does not exceed the cash
    on hand, so cash never becomes negative.
  * Reward r_t = (v_{t+1} - v_t) * reward_scale with v_t = b_t + p_t^T h_t
    (Section 3.1, Reward); v_t is the pre-trade value at p_t carried from the
    previous step and v_{t+1} uses the day t+1 close.  R accumulates r in
    step order (gamma = 1 in R(tau) of Section 4.3).
  * reset returns every sub-environment to day 0 with the initial cash and no
    holdings (Section 4.2, reset).  The market arrays hold T+1 days; the
    trajectory is done when the day index reaches T.
  * State order [b, p, h, f] (Section 3.1) with power-of-two scales:
    obs = [fl32(cash * 2^-20), p * 2^-8, fl32(h) * 2^-10, f (indicator-major)].
"""
from __future__ import annotations

import numpy as np

F64 = np.float64
F32 = np.float32


def orders(a, hmax: int) -> np.ndarray:
    """Integer share orders q = trunc(fl32(a * hmax)) for float32 actions a (any shape)."""
    a = np.asarray(a, dtype=F32)
    a = np.where(np.isnan(a), F32(0.0), np.clip(a, F32(-1.0), F32(1.0))).astype(F32)
    prod = (a * F32(hmax)).astype(F32)          # one float32 rounding
    return np.trunc(prod).astype(np.int32)


def buy_quantity(cash, price, q, one_p) -> np.ndarray:
    """Largest k in [0, q] with (price*k)*one_p <= cash, by exhaustive search.

    cash: float64 [N]; price: float scalar (float32 value); q: int [N] >= 0.
    Written as the definition: every candidate k = 0..max(q) is priced and the
    largest affordable one not above q is taken.
    """
    cash = np.asarray(cash, dtype=F64)
    q = np.asarray(q, dtype=np.int64)
    qmax = int(q.max()) if q.size else 0
    ks = np.arange(qmax + 1, dtype=F64)
    cost = (F64(price) * ks) * F64(one_p)                      # [qmax+1]
    ok = (cost[None, :] <= cash[:, None]) & (np.arange(qmax + 1)[None, :] <= q[:, None])
    # ok[:, 0] holds whenever cash >= 0; the largest True index is k.
    k = np.where(ok.any(axis=1), qmax - np.argmax(ok[:, ::-1], axis=1), 0)
    return k.astype(np.int32)


def execute_trades(cash, hold, price, q, cost_rate: float):
    """Sells then buys for every env, stocks in ascending order.

    cash float64 [N], hold int32 [N][D], price float32 [D], q int32 [N][D].
    Returns (cash', hold', executed) with executed int32 [N][D] signed
    (negative = shares sold).
    """
    cash = np.array(cash, dtype=F64, copy=True)
    hold = np.array(hold, dtype=np.int32, copy=True)
    q = np.asarray(q, dtype=np.int32)
    p = np.asarray(price, dtype=F32).astype(F64)
    one_m = F64(1.0) - F64(cost_rate)
    one_p = F64(1.0) + F64(cost_rate)
    n_envs, n_stocks = hold.shape
    executed = np.zeros((n_envs, n_stocks), dtype=np.int32)
    for d in range(n_stocks):                       # sells, ascending d
        sell = q[:, d] < 0
        s = np.where(sell, np.minimum(hold[:, d], -q[:, d]), 0).astype(np.int32)
        proceeds = (p[d] * s.astype(F64)) * one_m
        cash = np.where(sell, cash + proceeds, cash)
        hold[:, d] -= s
        executed[:, d] -= s
    for d in range(n_stocks):                       # buys, ascending d
        buy = q[:, d] > 0
        k = np.where(buy, buy_quantity(cash, p[d], np.maximum(q[:, d], 0), one_p), 0).astype(np.int32)
        debit = (p[d] * k.astype(F64)) * one_p
        cash = np.where(buy, cash - debit, cash)
        hold[:, d] += k
        executed[:, d] += k
    return cash, hold, executed


def portfolio_value(cash, hold, price) -> np.ndarray:
    """v = b + p^T h, accumulated in float64 in ascending stock order."""
    acc = np.array(cash, dtype=F64, copy=True)
    p = np.asarray(price, dtype=F32).astype(F64)
    hold = np.asarray(hold)
    for d in range(hold.shape[1]):
        acc = acc + p[d] * hold[:, d].astype(F64)
    return acc


class OracleEnv:
    """N sub-environments over one shared market (Section 4.2, VecEnv of SubEnvs)."""

    def __init__(self, cfg, close, ind, n_envs: int | None = None):
        self.cfg = cfg
        self.close = np.ascontiguousarray(close, dtype=F32)       # [T+1][D]
        self.ind = np.ascontiguousarray(ind, dtype=F32)           # [T+1][I][D]
        self.n_envs = int(cfg.n_envs if n_envs is None else n_envs)
        self.n_days = self.close.shape[0] - 1
        self.n_stocks = self.close.shape[1]
        if self.ind.shape[0] != self.n_days + 1 or self.ind.shape[2] != self.n_stocks:
            raise ValueError("indicator array does not match the close array")
        self.reset()

    # -- state -------------------------------------------------------------
    def reset(self) -> np.ndarray:
        """s_t -> s_0: day 0, initial cash, no holdings (Section 4.2, reset)."""
        n, d = self.n_envs, self.n_stocks
        self.day = 0
        self.cash = np.full(n, F64(self.cfg.init_cash))
        self.hold = np.zeros((n, d), dtype=np.int32)
        self.asset = portfolio_value(self.cash, self.hold, self.close[0])
        self.cumrew = np.zeros(n, dtype=F64)
        return self.obs()

    def obs(self) -> np.ndarray:
        """State [b, p, h, f] of Section 3.1 as float32 [N][(I+2)D+1]."""
        c = self.cfg
        n = self.n_envs
        cash = (self.cash * F64(c.cash_obs_scale)).astype(F32)[:, None]
        price = np.broadcast_to((self.close[self.day] * F32(c.price_obs_scale)).astype(F32),
                                (n, self.n_stocks))
        hold = (self.hold.astype(F32) * F32(c.hold_obs_scale)).astype(F32)
        feat = np.broadcast_to(self.ind[self.day].reshape(-1), (n, self.ind.shape[1] * self.n_stocks))
        return np.ascontiguousarray(np.concatenate([cash, price, hold, feat], axis=1), dtype=F32)

    def get_state(self):
        return dict(cash=self.cash.copy(), hold=self.hold.copy(), asset=self.asset.copy(),
                    cumrew=self.cumrew.copy(), day=int(self.day))

    def set_state(self, st):
        self.cash = np.array(st["cash"], dtype=F64)
        self.hold = np.array(st["hold"], dtype=np.int32)
        self.asset = np.array(st["asset"], dtype=F64)
        self.cumrew = np.array(st["cumrew"], dtype=F64)
        self.day = int(st["day"])

    # -- step / reward -----------------------------------------------------
    def step(self, actions):
        """(s_t, a_t) -> s_{t+1} and r_t (Section 4.2, step and reward).

        Returns (obs float32 [N][S], reward float64 [N], executed int32 [N][D], done).
        """
        if self.day >= self.n_days:
            raise RuntimeError("step past the last day; reset first")
        c = self.cfg
        q = orders(actions, c.hmax)
        self.cash, self.hold, executed = execute_trades(self.cash, self.hold, self.close[self.day], q,
                                                        c.cost_rate)
        self.day += 1
        v_new = portfolio_value(self.cash, self.hold, self.close[self.day])
        reward = (v_new - self.asset) * F64(c.reward_scale)
        self.cumrew = self.cumrew + reward
        self.asset = v_new
        return self.obs(), reward, executed, self.day == self.n_days
