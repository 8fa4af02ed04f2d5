"""Uneven batch of environment groups: stock counts, environment counts, horizons and market
volatility drawn per group (the batched form of the vectorised environment)."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .configs import ActorConfig, EnvConfig, state_width


@dataclass(frozen=True)
class UnevenGroup:
    env: EnvConfig
    actors: ActorConfig
    market_seed: int
    vol: float


def uneven_groups(seed: int = 4, n_groups: int = 64, d_choices=(5, 10, 30, 50, 100), n_range=(32, 4096),
                  t_range=(20, 1000), vol_range=(0.01, 0.04), hidden: int = 256, n_ind: int = 5):
    """Groups with D uniform over d_choices, N log-uniform over n_range, T uniform over t_range
    (inclusive), per-group GBM volatility uniform over vol_range; K=3 actors (7D+1)->H->H->D."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n_groups):
        D = int(rng.choice(np.asarray(d_choices)))
        N = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        T = int(rng.integers(t_range[0], t_range[1] + 1))
        vol = float(rng.uniform(*vol_range))
        S = state_width(D, n_ind)
        out.append(UnevenGroup(EnvConfig(n_envs=N, n_stocks=D, n_ind=n_ind, n_days=T),
                               ActorConfig(n_actors=3, in_dim=S, hidden=hidden, out_dim=D, seed_base=3000 + 10 * g),
                               market_seed=5000 + g, vol=vol))
    return out
