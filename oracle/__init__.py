"""CPU oracle for the massively parallel trading-environment rollout.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The library's GPU
path never calls it and shares no code with it.

Plain, slow, float64 numpy code written from the paper:
  * env.py     -- the MDP of Section 3.1 (state [b, p, h, f], share-change
                  actions, reward v_{t+1} - v_t with v_t = b_t + p_t^T h_t)
                  and the reset / step / reward operations of Section 4.2.
  * philox.py  -- Philox4x64-10 (Salmon et al., SC'11) and the Box-Muller
                  map used for Gaussian action noise.
  * policy.py  -- the K-actor MLP forward and the stock ensemble rule of
                  Section 5.2.1 (weighted average of the agents' actions).
  * rollout.py -- T-step trajectories (Section 4.3, the T x N x D sample
                  tensors and R(tau) = sum_t gamma^t r_t).
  * metrics.py -- backtest metrics (Section 6.1), softmax-of-Sharpe weights and
                  the majority vote (Section 5.2).
  * learner.py -- the consumer of the samples: the Monte-Carlo policy gradient
                  of eq. (4) with the agent-diversity KL term of eq. (5).
  * crypto.py  -- the single-asset crypto task: discrete target positions with a
                  proportional fee, the agents' Q-networks, the averaged-softmax
                  and majority-vote ensemble rules, exploration draws and the
                  running backtest statistics (Sections 3.1, 5.2.2, 6.1).

Each function is vectorised over environments only; loops over stocks run in
ascending order so every environment's floating-point operation order is the
literal one.  Every function here is pinned by the CPU tests against hand-worked
examples, invariants, brute force or a library routine (see tests/).
"""
from .env import OracleEnv, orders, execute_trades, portfolio_value, buy_quantity
from .philox import philox4x64_10, uniforms_from_words, box_muller, noise
from .policy import actor_forward, ensemble_mean, ensemble_act, round_to_bf16
from .rollout import rollout_closed_loop, rollout_driven

__all__ = [
    "OracleEnv", "orders", "execute_trades", "portfolio_value", "buy_quantity",
    "philox4x64_10", "uniforms_from_words", "box_muller", "noise",
    "actor_forward", "ensemble_mean", "ensemble_act", "round_to_bf16",
    "rollout_closed_loop", "rollout_driven",
]
