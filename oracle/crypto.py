"""Oracle for the single-asset crypto task (TEST INFRASTRUCTURE ONLY; see the package docstring).

The crypto task of Sections 3.1 and 5.2.2 trades one asset with a discrete action space.  The
readings taken here, in the paper's notation:

  * State s_t = [b_t, p_t, h_t, f_t] (Section 3.1, State) with one asset: the cash b, the mid price
    p, the position h and 13 market features f (the tick table's columns 3..15).  The actor sees
    x = fl32([b 2^-17, p 2^-16, h, f]); the power-of-two scales are exact, so the only rounding is
    the one conversion to float32.
  * Actions (Section 5.2.2) are discrete: action j in {0, 1, 2} sets the position to h' = j - 1
    (short one unit, flat, long one unit).  The trade of Delta = h' - h units happens at the tick's
    mid price p and costs a fee proportional to its notional: b' = (b - Delta p) - (|Delta| p) fee.
  * Reward (Section 3.1, Reward): r_t = v_{t+1} - v_t with v = b + h p, the position marked at the
    next tick's mid price.
  * Agents (Section 6.1: DQN-family networks, here 16 -> 128 -> 128 -> 3) output three Q-values
    through ReLU hidden layers.  Ensemble rules: the average over agents of softmax(Q) with weights
    w_k (1/K by default), the action being its argmax with ties to the lowest index; or the
    majority vote of the agents' own argmax actions (Section 5.2.2), ties to the lowest action.
  * Exploration: with probability eps the action is replaced by a uniformly random one.  The draws
    come from Philox4x64-10 with key (request key, 1) and counter (n, t, 0, 0), n being the
    environment's index inside its request: word 0 gives u = ((w0 >> 41) + 0.5) 2^-23 and the
    environment explores iff u < eps (eps as float32); the random action is (w1 >> 32) mod 3.
  * Running backtest statistics per environment (Section 6.1 metrics are formed from them):
    sum of r, sum of r^2, running peak of v and the largest drawdown peak - v, in dollars, and the
    number of ticks on which the position changed.

All arithmetic is float64 numpy in the order written; the bfloat16 reading of the stock oracle
applies to the weights (the oracle evaluates the device's bfloat16-rounded weight matrices).
"""
from __future__ import annotations

import numpy as np

from .metrics import majority_vote
from .philox import U64, philox4x64_10, uniforms_from_words

CASH_SCALE = 2.0 ** -17
PRICE_SCALE = 2.0 ** -16
AVG_SOFTMAX, MAJORITY_VOTE = 0, 1


def state_rows(cash, pos, mid, feat_rows) -> np.ndarray:
    """x = fl32([b 2^-17, p 2^-16, h, f]) for every environment: float32 [n][16]."""
    x = np.array(feat_rows, dtype=np.float32, copy=True)
    x[:, 0] = (np.asarray(cash, np.float64) * CASH_SCALE).astype(np.float32)
    x[:, 1] = (np.asarray(mid, np.float64) * PRICE_SCALE).astype(np.float32)
    x[:, 2] = np.asarray(pos).astype(np.float32)
    return x


def q_values(p, x) -> np.ndarray:
    """Q = relu(relu(x W1 + b1) W2 + b2) W3 + b3 in float64; x [n][16] -> [n][3]."""
    h = np.asarray(x, dtype=np.float64)
    h = np.maximum(h @ np.asarray(p["W1"], np.float64) + np.asarray(p["b1"], np.float64), 0.0)
    h = np.maximum(h @ np.asarray(p["W2"], np.float64) + np.asarray(p["b2"], np.float64), 0.0)
    return h @ np.asarray(p["W3"], np.float64) + np.asarray(p["b3"], np.float64)


def softmax(q) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    e = np.exp(q - q.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def ensemble_probs(actors, x, mix=None) -> np.ndarray:
    """sum_k w_k softmax(Q_k(x)), summed in ascending k: float64 [n][3]."""
    K = len(actors)
    w = np.full(K, 1.0 / K) if mix is None else np.asarray(mix, dtype=np.float32).astype(np.float64)
    acc = None
    for k, p in enumerate(actors):
        term = w[k] * softmax(q_values(p, x))
        acc = term if acc is None else acc + term
    return acc


def first_argmax(v) -> np.ndarray:
    """Index of the largest entry along the last axis, the lowest index among equal ones."""
    return np.argmax(np.asarray(v), axis=-1)


def vote_actions(actors, x) -> np.ndarray:
    """Majority vote of the agents' argmax actions (Section 5.2.2)."""
    return majority_vote(np.stack([first_argmax(q_values(p, x)) for p in actors]), 3)


def exploration(key: int, env_idx, t: int, eps: float):
    """(explore mask, random action) for environments env_idx of a request at step t."""
    env_idx = np.asarray(env_idx, dtype=U64)
    ctr = np.zeros((env_idx.size, 4), dtype=U64)
    ctr[:, 0] = env_idx
    ctr[:, 1] = U64(t)
    w = philox4x64_10(ctr, np.array([key, 1], dtype=U64))
    u = uniforms_from_words(w[:, 0])
    explore = u < np.float64(np.float32(eps))
    rand = ((w[:, 1] >> U64(32)) % U64(3)).astype(np.int64)
    return explore, rand


def trade(cash, pos, price, action, fee: float):
    """Move to position action - 1 at the given price: (cash', pos', changed)."""
    new_pos = np.asarray(action, dtype=np.int64) - 1
    delta = new_pos - np.asarray(pos, dtype=np.int64)
    p = np.asarray(price, dtype=np.float64)
    cash1 = (np.asarray(cash, np.float64) - delta.astype(np.float64) * p) - (np.abs(delta).astype(np.float64) * p) * fee
    return cash1, new_pos, delta != 0


class CryptoState:
    """Per-environment state of one request: cash, position, value and the running statistics."""

    def __init__(self, n: int, cash0: float):
        self.cash = np.full(n, cash0, dtype=np.float64)
        self.pos = np.zeros(n, dtype=np.int64)
        self.value = np.full(n, cash0, dtype=np.float64)
        self.sum_r = np.zeros(n, dtype=np.float64)
        self.sum_r2 = np.zeros(n, dtype=np.float64)
        self.peak = np.full(n, cash0, dtype=np.float64)
        self.mdd = np.zeros(n, dtype=np.float64)
        self.trades = np.zeros(n, dtype=np.int64)

    def as_dict(self):
        return {k: getattr(self, k).copy() for k in
                ("cash", "pos", "value", "sum_r", "sum_r2", "peak", "mdd", "trades")}


def step(st: CryptoState, action, price, next_price, fee: float):
    """One tick for every environment of st: trade, mark to the next price, update statistics.
    Returns the rewards."""
    cash1, pos1, changed = trade(st.cash, st.pos, price, action, fee)
    v1 = cash1 + pos1.astype(np.float64) * np.asarray(next_price, np.float64)
    r = v1 - st.value
    st.sum_r = st.sum_r + r
    st.sum_r2 = st.sum_r2 + r * r
    st.peak = np.maximum(st.peak, v1)
    st.mdd = np.maximum(st.mdd, st.peak - v1)
    st.trades = st.trades + changed.astype(np.int64)
    st.cash, st.pos, st.value = cash1, pos1, v1
    return r


def env_ticks(start_tick: int, stride: int, n_envs: int, t: int) -> np.ndarray:
    """Tick index of every environment of a request at step t."""
    return start_tick + stride * np.arange(n_envs, dtype=np.int64) + t


def rollout(market, actors, n_envs: int, horizon: int, start_tick: int, stride: int, key: int, eps: float,
            fee: float = 2e-4, cash0: float = 1e5, mode: int = AVG_SOFTMAX, mix=None, actions=None,
            obs_out=None):
    """A request's trajectories.  Closed loop unless actions [horizon][n] is given, in which case
    the environment is driven by those actions and the policy is still evaluated on the states the
    environment reaches.  Returns (final state dict, probs [T][n][3] (average mode), chosen
    actions [T][n], per-step decided-by-policy actions [T][n], explore mask [T][n], rewards [T][n]).
    obs_out, if given, is a list that receives each step's state rows."""
    st = CryptoState(n_envs, cash0)
    T = horizon
    probs = np.zeros((T, n_envs, 3))
    chosen = np.zeros((T, n_envs), dtype=np.int64)
    greedy = np.zeros((T, n_envs), dtype=np.int64)
    explored = np.zeros((T, n_envs), dtype=bool)
    rew = np.zeros((T, n_envs))
    idx = np.arange(n_envs)
    for t in range(T):
        ticks = env_ticks(start_tick, stride, n_envs, t)
        x = state_rows(st.cash, st.pos, market.mid[ticks], market.feat[ticks])
        if obs_out is not None:
            obs_out.append(x)
        if mode == AVG_SOFTMAX:
            probs[t] = ensemble_probs(actors, x, mix)
            greedy[t] = first_argmax(probs[t])
        else:
            greedy[t] = vote_actions(actors, x)
        explored[t], rand = exploration(key, idx, t, eps)
        chosen[t] = np.where(explored[t], rand, greedy[t])
        act = chosen[t] if actions is None else np.asarray(actions[t], dtype=np.int64)
        rew[t] = step(st, act, market.mid[ticks], market.mid[ticks + 1], fee)
    return st.as_dict(), probs, chosen, greedy, explored, rew
