"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generation only (market paths, technical indicators,
actor weight initialisation, action tensors, workload sizes).  It contains none
of the trading environment's or the ensemble's arithmetic, so that the CPU
oracle and the GPU path can both consume it without sharing any of the method.

The paper trains on daily OHLCV of the 30 Dow Jones stocks (Section 6.1) and
measures sampling speed on them (Section 6.2).  Those records are not
available here; the generators below produce inputs of the same shape
(30 stocks, daily steps, one trading year of 252 days) from a seeded
geometric Brownian motion instead.
"""
from .configs import (EnvConfig, ActorConfig, Workload, WORKLOADS, TINY, PAPER_SCALE,
                      PRECISION, state_width)
from .market import Market, make_market
from .actors import make_actor_weights, pack_actor_weights, unpack_actor_weights
from .actions import make_actions

__all__ = [
    "EnvConfig", "ActorConfig", "Workload", "WORKLOADS", "TINY", "PAPER_SCALE", "PRECISION",
    "state_width", "Market", "make_market", "make_actor_weights", "pack_actor_weights",
    "unpack_actor_weights", "make_actions",
]
