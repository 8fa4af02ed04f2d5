"""Seeded inputs for the single-asset crypto task and its serving workload.

The paper's crypto task trades one asset (BTC) from second-level limit-order-book data with
indicators derived by a recurrent network (Sections 3.1 and 6.1).  Those records are not
available here; this module generates a tick series of the same kind instead:

  * log returns r_t drawn from a Student-t with 3 degrees of freedom, divided by sqrt(3) (the
    standard deviation of that distribution) and scaled to 1e-4 per tick; mid_t = mid_0 exp(sum r);
  * 13 market features per tick, all from data up to and including tick t: the last 10 returns,
    rolling standard deviations of the returns over 10 and 60 ticks (all x 1e4), and a synthetic
    order-book imbalance drawn uniformly from [-1, 1].

The feature table has 16 float32 columns per tick; columns 0-2 are left at zero because the
agent's state puts its cash, the price and its position there.  Requests of the serving
workload arrive as a Poisson process; their environment counts and horizons are log-uniform.
Nothing here is part of the trading or policy arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .configs import ActorConfig

N_FEAT = 16          # columns of the feature table (and the actors' input width)
N_MARKET = 13        # market features, in columns 3..15
N_LAGS = 10
VOL_WINDOWS = (10, 60)
WARMUP = 64          # first tick whose features are all defined


@dataclass(frozen=True)
class TickMarket:
    mid: np.ndarray    # float64 [n_ticks]
    feat: np.ndarray   # float32 [n_ticks][16]; columns 0..2 zero

    @property
    def n_ticks(self) -> int:
        return int(self.mid.shape[0])


def _rolling_std(r: np.ndarray, w: int) -> np.ndarray:
    """Population standard deviation of r[t-w+1..t] for t >= w-1 (zero before)."""
    c1 = np.concatenate([[0.0], np.cumsum(r)])
    c2 = np.concatenate([[0.0], np.cumsum(r * r)])
    out = np.zeros_like(r)
    s1 = c1[w:] - c1[:-w]
    s2 = c2[w:] - c2[:-w]
    var = np.maximum(s2 / w - (s1 / w) ** 2, 0.0)
    out[w - 1:] = np.sqrt(var)
    return out


def make_ticks(seed: int = 11, n_ticks: int = 1_000_000, mid0: float = 50_000.0, scale: float = 1e-4) -> TickMarket:
    rng = np.random.default_rng(seed)
    r = rng.standard_t(3, size=n_ticks) / math.sqrt(3.0) * scale
    r[0] = 0.0
    mid = mid0 * np.exp(np.cumsum(r))
    feat = np.zeros((n_ticks, N_FEAT), dtype=np.float64)
    for i in range(N_LAGS):
        feat[i:, 3 + i] = r[:n_ticks - i] * 1e4
    for j, w in enumerate(VOL_WINDOWS):
        feat[:, 3 + N_LAGS + j] = _rolling_std(r, w) * 1e4
    feat[:, 15] = rng.uniform(-1.0, 1.0, size=n_ticks)
    return TickMarket(mid=mid.astype(np.float64), feat=feat.astype(np.float32))


def crypto_actors(n_actors: int = 5, hidden: int = 128, seed_base: int = 7000, bias_std: float = 0.05) -> ActorConfig:
    """K actors 16 -> H -> H -> 3 (Q-values of the three target positions)."""
    return ActorConfig(n_actors=n_actors, in_dim=N_FEAT, hidden=hidden, out_dim=3, seed_base=seed_base,
                       bias_std=bias_std)


def make_crypto_agents(cfg: ActorConfig, q_gain: float = 4.0):
    """Seeded agents (Xavier initialisation) with the output layer scaled by q_gain, so that the
    three action values differ by O(1) and the ensemble's decisions are not all near-ties."""
    from .actors import make_actor_weights
    agents = make_actor_weights(cfg)
    for a in agents:
        a["W3"] = (a["W3"] * np.float32(q_gain)).astype(np.float32)
    return agents


@dataclass(frozen=True)
class CryptoRequest:
    arrival_s: float     # arrival time from the start of the run
    n_envs: int
    horizon: int         # ticks per environment
    start_tick: int      # first tick of environment 0
    stride: int          # environment n starts at start_tick + n * stride
    key: int             # exploration stream


def place(rng: np.random.Generator, n_envs: int, horizon: int, n_ticks: int):
    """A start tick and stride such that every environment's window [start, start + horizon] lies
    inside the defined part of the tick table."""
    room = n_ticks - 1 - WARMUP - horizon
    if room < 0:
        raise ValueError("horizon longer than the tick table")
    stride = 0 if n_envs == 1 else int(rng.integers(0, min(257, room // (n_envs - 1) + 1)))
    span = stride * (n_envs - 1)
    start = WARMUP + int(rng.integers(0, room - span + 1))
    return start, stride


def poisson_requests(seed: int, n_requests: int, rate_per_s: float, n_ticks: int, n_range=(1, 4096),
                     horizon_range=(1000, 100_000)):
    """Poisson arrivals at rate_per_s; environment counts and horizons log-uniform over the ranges."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        h = int(round(math.exp(rng.uniform(math.log(horizon_range[0]), math.log(horizon_range[1])))))
        start, stride = place(rng, n, h, n_ticks)
        out.append(CryptoRequest(arrival_s=t, n_envs=n, horizon=h, start_tick=start, stride=stride,
                                 key=0x5EED0000 + i))
    return out
