"""Seeded action tensors for driven-mode rollouts (actions supplied by the caller).

The mix covers every branch of the order logic: exact zeros, values that
truncate to zero orders, sells larger than the holding, buys that exhaust
cash, the clip boundaries +-1 and values just inside them.
"""
from __future__ import annotations

import numpy as np


def make_actions(seed: int, n_steps: int, n_envs: int, n_stocks: int, buy_bias: float = 0.15,
                 dtype=np.float32) -> np.ndarray:
    """float32 [T][N][D] actions in [-1, 1] with a mix of special values."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(n_steps, n_envs, n_stocks)) + buy_bias
    u = rng.uniform(size=a.shape)
    a = np.where(u < 0.05, 0.0, a)
    a = np.where((u >= 0.05) & (u < 0.10), rng.uniform(-0.0099, 0.0099, size=a.shape), a)
    a = np.where((u >= 0.10) & (u < 0.12), 1.0, a)
    a = np.where((u >= 0.12) & (u < 0.14), -1.0, a)
    a = np.clip(a, -1.0, 1.0)
    return np.ascontiguousarray(a, dtype=dtype)
