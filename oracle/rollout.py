"""T-step trajectories (TEST INFRASTRUCTURE ONLY; see the package docstring).

Section 4.3 stores the samples as T x N x D tensors of states, actions and
rewards; a trajectory is (s_0, a_1, s_1, ..., s_T) and its return is
R(tau) = sum_t gamma^t r_t (gamma = 1 here).
"""
from __future__ import annotations

import numpy as np

from .env import OracleEnv
from .policy import ensemble_act


def rollout_driven(cfg, close, ind, actions, n_envs=None):
    """Replay caller-supplied float32 actions [T][N][D].

    Returns dict with obs [T+1][N][S] (obs[0] = s_0), exec [T][N][D],
    reward [T][N], and the final cash, hold, asset, cumrew, day.
    """
    actions = np.asarray(actions, dtype=np.float32)
    T, N, _ = actions.shape
    env = OracleEnv(cfg, close, ind, n_envs=N if n_envs is None else n_envs)
    obs = [env.reset()]
    ex, rw = [], []
    for t in range(T):
        o, r, x, _ = env.step(actions[t])
        obs.append(o)
        ex.append(x)
        rw.append(r)
    out = dict(obs=np.stack(obs), exec=np.stack(ex), reward=np.stack(rw))
    out.update(env.get_state())
    return out


def rollout_closed_loop(cfg, close, ind, actors, n_steps, sigma, noise_key, mix=None, n_envs=None):
    """The ensemble acts on each state, then the environment steps (producer half of Section 3.2)."""
    env = OracleEnv(cfg, close, ind, n_envs=n_envs)
    o = env.reset()
    obs, acts, ex, rw = [o], [], [], []
    for t in range(n_steps):
        a = ensemble_act(actors, o, t, 0, sigma, noise_key, mix)
        o, r, x, _ = env.step(a)
        acts.append(a)
        obs.append(o)
        ex.append(x)
        rw.append(r)
    out = dict(obs=np.stack(obs), act=np.stack(acts), exec=np.stack(ex), reward=np.stack(rw))
    out.update(env.get_state())
    return out
