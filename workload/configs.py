"""Workload sizes for the trading-environment rollout.

Symbols follow the paper's MDP (Section 3.1): the state is
[balance, prices, holdings, features] with width (I+2)*D+1, where D is the
number of stocks and I the number of technical indicators per stock.  The
paper writes K for the number of assets; here K is the number of actors in
the ensemble and D the number of stocks.
"""
from __future__ import annotations

import dataclasses


def state_width(n_stocks: int, n_ind: int) -> int:
    """Width of the MDP state [b, p, h, f]: (I+2)*D+1 (Section 3.1, State)."""
    return (n_ind + 2) * n_stocks + 1


@dataclasses.dataclass(frozen=True)
class EnvConfig:
    n_envs: int = 16          # N parallel sub-environments (Section 4.2)
    n_stocks: int = 30        # D assets (30 Dow Jones stocks, Section 3.1)
    n_ind: int = 5            # I indicators per stock
    n_days: int = 30          # T steps per trajectory; market arrays hold T+1 days
    hmax: int = 100           # shares per unit action
    init_cash: float = 1e6
    cost_rate: float = 1e-3   # proportional transaction cost (Section 3.2 constraints)
    reward_scale: float = 2.0 ** -12
    cash_obs_scale: float = 2.0 ** -20
    price_obs_scale: float = 2.0 ** -8
    hold_obs_scale: float = 2.0 ** -10

    @property
    def state_dim(self) -> int:
        return state_width(self.n_stocks, self.n_ind)

    def replace(self, **kw) -> "EnvConfig":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass(frozen=True)
class ActorConfig:
    n_actors: int = 3         # K actors in the ensemble (Section 5.2.1: PPO, SAC, DDPG)
    in_dim: int = 211         # S
    hidden: int = 64          # H
    out_dim: int = 30         # A = D (one action per stock)
    seed_base: int = 2000     # actor k uses seed_base + k
    bias_std: float = 0.0     # Xavier init keeps biases at zero; tests draw nonzero ones

    def replace(self, **kw) -> "ActorConfig":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    env: EnvConfig
    actors: ActorConfig
    market_seed: int = 1001
    noise_key: int = 7
    sigma: float = 0.1
    dtype: str = "f32"


_S = state_width(30, 5)

# Tiny case: 16 envs, 30 stocks, 30 days, three 211->64->64->30 actors.
TINY = Workload("tiny N=16 D=30 T=30 H=64", EnvConfig(n_envs=16, n_days=30),
                ActorConfig(in_dim=_S, hidden=64, out_dim=30), sigma=0.1, dtype="f32")
# Paper scale: 2048 envs (the paper's largest sampling-speed point, Section 6.2),
# 30 stocks, one trading year of 252 days, three 211->256->256->30 actors.
PAPER_SCALE = Workload("paper-scale N=2048 D=30 T=252 H=256", EnvConfig(n_envs=2048, n_days=252),
                       ActorConfig(in_dim=_S, hidden=256, out_dim=30), sigma=0.1, dtype="f32")
# Precision form: the same actors in BF16 on 8192 envs.
PRECISION = Workload("precision N=8192 D=30 T=252 H=256 bf16", EnvConfig(n_envs=8192, n_days=252),
                     ActorConfig(in_dim=_S, hidden=256, out_dim=30), sigma=0.1, dtype="bf16")

# Environment-kernel throughput: enough environments to fill the GPU many times over, fewer days
# (the driven trajectories of 65536 x 64 steps are 3.5 GB of states).
ENV_LARGE = Workload("env-throughput N=65536 D=30 T=64", EnvConfig(n_envs=65536, n_days=64),
                     ActorConfig(in_dim=_S, hidden=256, out_dim=30), sigma=0.1, dtype="f32")

WORKLOADS = {"tiny": TINY, "paper": PAPER_SCALE, "precision": PRECISION, "envlarge": ENV_LARGE}
