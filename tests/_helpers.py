"""Shared helpers for the GPU parity tests (the GPU path against the CPU oracle)."""
from __future__ import annotations

import numpy as np

from oracle.policy import device_weights, ensemble_act
from oracle.rollout import rollout_driven
from workload import ActorConfig, EnvConfig, make_actor_weights, make_market, pack_actor_weights

# Tolerances on actions (absolute): float32 path and bfloat16 path against the float64 oracle.
TOL_F32 = 1e-5
TOL_BF16 = 2e-2
# float64 accounting (cash, total asset, rewards): relative.
TOL_F64_REL = 1e-12


def cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU")
    return torch.device("cuda:0")


def env_case(N, D, I, T, seed, hmax=100, cash=1e6, cost=1e-3):
    cfg = EnvConfig(n_envs=N, n_stocks=D, n_ind=I, n_days=T, hmax=hmax, init_cash=cash, cost_rate=cost)
    m = make_market(seed, D, T, n_ind=I)
    return cfg, m


def actors_case(K, S, H, A, bias_std=0.1, seed_base=2000):
    acfg = ActorConfig(n_actors=K, in_dim=S, hidden=H, out_dim=A, bias_std=bias_std, seed_base=seed_base)
    actors = make_actor_weights(acfg)
    return acfg, actors, pack_actor_weights(actors)


def assert_f64_close(got, want, scale, what):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    err = np.abs(got - want)
    bound = TOL_F64_REL * np.maximum(np.abs(scale), 1.0)
    bad = err > bound
    assert not bad.any(), f"{what}: {bad.sum()} values off, worst {err.max():.3e}"


def check_replay(cfg, m, traj, obs0, env_ids=None):
    """Replay the GPU's executed actions through the oracle; the environment must agree exactly.

    traj: dict of numpy arrays act [T][N][D], obs [T][N][S], rew [T][N], qty [T][N][D].
    env_ids: subset of environments to check (default all).
    """
    act = traj["act"]
    ids = np.arange(act.shape[1]) if env_ids is None else np.asarray(env_ids)
    ref = rollout_driven(cfg.replace(n_envs=len(ids)), m.close, m.ind, act[:, ids, :])
    assert np.array_equal(obs0[ids], ref["obs"][0]), "s_0 differs"
    assert np.array_equal(traj["qty"][:, ids], ref["exec"]), "executed quantities differ"
    assert np.array_equal(traj["obs"][:, ids], ref["obs"][1:]), "states differ"
    # r = (v' - v) * scale cancels, so its error is bounded relative to |v| + |v'|.
    v_scale = 2.0 * max(cfg.init_cash, float(np.abs(ref["asset"]).max()))
    err = np.abs(traj["rew"][:, ids] - ref["reward"])
    assert np.all(err <= TOL_F64_REL * 2 * v_scale * cfg.reward_scale), f"rewards off by {err.max():.3e}"
    return ref


def check_actions(actors, dtype, traj, obs0, sigma, key, tol, env_ids=None, steps=None, env_offset=0,
                  id_map=None):
    """The GPU's action at (t, n) against the oracle ensemble acting on the GPU's own state s_t.

    env_ids / steps select a sample (default all).  id_map: global environment index of each
    column of traj when traj holds a subset of the batch.  Returns the largest absolute error.
    """
    w = device_weights(actors, dtype)
    act = traj["act"]
    T, N, _ = act.shape
    ids = np.arange(N) if env_ids is None else np.asarray(env_ids)
    glob = ids if id_map is None else np.asarray(id_map)[ids]
    worst = 0.0
    for t in (range(T) if steps is None else steps):
        s_t = obs0[ids] if t == 0 else traj["obs"][t - 1][ids]
        a_ref = ensemble_act(w, s_t, t, 0, sigma, key, env_ids=env_offset + glob)
        e = float(np.max(np.abs(a_ref.astype(np.float64) - act[t][ids].astype(np.float64))))
        worst = max(worst, e)
    assert worst <= tol, f"actions off by {worst:.3e} (tolerance {tol})"
    return worst
