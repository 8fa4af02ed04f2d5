"""Thin ctypes binding of libfinrl_mi.so (include/finrl_mi.h).

The functions below carry the C entry points' names and only marshal arguments: torch
tensors become device pointers, the current torch stream becomes the hipStream_t, and a
non-OK status becomes an exception carrying fm_last_error().  All computation happens in the
library's HIP kernels; if the library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfinrl_mi.so")

FM_OK, FM_ERR_INVALID, FM_ERR_STATE, FM_ERR_DEVICE, FM_ERR_UNSUPPORTED = range(5)
FM_F32, FM_BF16 = 0, 1
FM_PATH_PLAIN, FM_PATH_FUSED = 0, 1

# Symbols declared in include/finrl_mi.h.
EXPORTS = (
    "env_workspace_bytes", "env_create", "env_reset", "env_step", "env_rollout", "env_read_state",
    "env_write_state", "env_day", "env_set_tile", "env_set_step_kernel", "env_set_fused_tuning", "env_destroy", "ensemble_workspace_bytes", "ensemble_create",
    "ensemble_act", "ensemble_destroy", "fm_last_error", "fm_noise", "fm_version", "fm_backtest_metrics",
    "fm_sharpe_weights", "fm_batch_workspace_bytes", "fm_batch_create", "fm_batch_tune", "fm_batch_set_tiling",
    "fm_batch_run",
    "fm_batch_destroy", "fm_serve_request_bytes", "fm_serve_workspace_bytes", "fm_serve_create", "fm_serve_submit",
    "fm_serve_step", "fm_serve_poll", "fm_serve_destroy", "fm_pg_workspace_bytes", "fm_policy_gradient",
    "fm_policy_gradient_noalloc",
)
FM_RULE_AVG_SOFTMAX, FM_RULE_MAJORITY_VOTE = 0, 1


class FmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"finrl_mi status {status}: {msg}")
        self.status = status


class FmEnvConfig(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32), ("n_stocks", ctypes.c_int32), ("n_ind", ctypes.c_int32),
        ("n_days", ctypes.c_int32), ("hmax", ctypes.c_int32),
        ("init_cash", ctypes.c_double), ("cost_rate", ctypes.c_double), ("reward_scale", ctypes.c_double),
        ("cash_obs_scale", ctypes.c_float), ("price_obs_scale", ctypes.c_float),
        ("hold_obs_scale", ctypes.c_float),
    ]


class FmRolloutOpts(ctypes.Structure):
    _fields_ = [
        ("d_actions", ctypes.c_void_p), ("sigma", ctypes.c_float), ("noise_key", ctypes.c_uint64),
        ("env_offset", ctypes.c_int64), ("path", ctypes.c_int32),
        ("d_obs_traj", ctypes.c_void_p), ("d_act_traj", ctypes.c_void_p),
        ("d_rew_traj", ctypes.c_void_p), ("d_qty_traj", ctypes.c_void_p),
    ]


class FmCryptoResult(ctypes.Structure):
    _fields_ = [("cash", ctypes.c_double), ("value", ctypes.c_double), ("sum_r", ctypes.c_double),
                ("sum_r2", ctypes.c_double), ("peak", ctypes.c_double), ("max_drawdown", ctypes.c_double),
                ("position", ctypes.c_int32), ("trades", ctypes.c_int32), ("ticks", ctypes.c_int64)]


class FmServeConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("d_mid", ctypes.c_void_p), ("d_feat", ctypes.c_void_p),
                ("n_ticks", ctypes.c_int64), ("n_agents", ctypes.c_int32), ("h_weights", ctypes.c_void_p),
                ("h_mix", ctypes.c_void_p), ("rule", ctypes.c_int32), ("eps", ctypes.c_float),
                ("fee", ctypes.c_double), ("cash0", ctypes.c_double), ("tile_rows", ctypes.c_int32),
                ("chunk_ticks", ctypes.c_int32), ("max_requests", ctypes.c_int32),
                ("max_active_envs", ctypes.c_int64), ("grid", ctypes.c_int32), ("d_pool", ctypes.c_void_p),
                ("pool_bytes", ctypes.c_size_t), ("d_workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class FmServeRequest(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("stride", ctypes.c_int32), ("horizon", ctypes.c_int64),
                ("start_tick", ctypes.c_int64), ("key", ctypes.c_uint64), ("d_result", ctypes.c_void_p),
                ("d_act", ctypes.c_void_p), ("d_prob", ctypes.c_void_p)]


class FmBatchGroup(ctypes.Structure):
    _fields_ = [("env", ctypes.c_void_p), ("ens", ctypes.c_void_p), ("n_steps", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("noise_key", ctypes.c_uint64), ("env_offset", ctypes.c_int64),
                ("d_obs_traj", ctypes.c_void_p), ("d_act_traj", ctypes.c_void_p), ("d_rew_traj", ctypes.c_void_p),
                ("d_qty_traj", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime under the same soname; importing it first makes the library
    # bind to that runtime, so the process holds one runtime and torch's pointers and streams are
    # valid in the library's calls.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "env_workspace_bytes": (SZ, [ctypes.POINTER(FmEnvConfig)]),
        "env_create": (I32, [ctypes.POINTER(FmEnvConfig), P, P, P, SZ, P, ctypes.POINTER(P)]),
        "env_reset": (I32, [P, P]),
        "env_step": (I32, [P, P, P, P, P, ctypes.POINTER(I32)]),
        "env_rollout": (I32, [P, P, I32, ctypes.POINTER(FmRolloutOpts)]),
        "env_read_state": (I32, [P, P, P, P, P, ctypes.POINTER(I32)]),
        "env_write_state": (I32, [P, P, P, P, P, I32]),
        "env_day": (I32, [P]),
        "env_set_tile": (I32, [P, I32, ctypes.POINTER(I32)]),
        "env_set_step_kernel": (I32, [P, I32, I32]),
        "env_set_fused_tuning": (I32, [P, I32, I32, I32]),
        "env_destroy": (None, [P]),
        "ensemble_workspace_bytes": (SZ, [I32, I32, I32, I32, I32, I32]),
        "ensemble_create": (I32, [I32, I32, I32, I32, I32, P, P, I32, P, SZ, P, ctypes.POINTER(P)]),
        "ensemble_act": (I32, [P, P, I32, ctypes.c_float, U64, I32, I64, P, P, P]),
        "ensemble_destroy": (None, [P]),
        "fm_last_error": (ctypes.c_char_p, []),
        "fm_noise": (I32, [U64, I64, I32, I32, I32, P, P, P]),
        "fm_version": (ctypes.c_char_p, []),
        "fm_backtest_metrics": (I32, [P, I32, I32, ctypes.c_double, P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, P, P]),
        "fm_sharpe_weights": (I32, [P, I32, ctypes.c_double, P]),
        "fm_batch_workspace_bytes": (SZ, [ctypes.POINTER(FmBatchGroup), I32]),
        "fm_batch_create": (I32, [ctypes.POINTER(FmBatchGroup), I32, P, SZ, P, ctypes.POINTER(P)]),
        "fm_batch_tune": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "fm_batch_set_tiling": (I32, [P, I32, I32]),
        "fm_batch_run": (I32, [P, I32]),
        "fm_batch_destroy": (None, [P]),
        "fm_serve_request_bytes": (SZ, [I32]),
        "fm_serve_workspace_bytes": (SZ, [ctypes.POINTER(FmServeConfig)]),
        "fm_serve_create": (I32, [ctypes.POINTER(FmServeConfig), P, ctypes.POINTER(P)]),
        "fm_serve_submit": (I32, [P, ctypes.POINTER(FmServeRequest), ctypes.POINTER(I64)]),
        "fm_serve_step": (I32, [P, P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "fm_serve_poll": (I32, [P, I32, ctypes.POINTER(I64), I32, ctypes.POINTER(I32)]),
        "fm_serve_destroy": (None, [P]),
        "fm_pg_workspace_bytes": (SZ, [I32, I32, I32, I32, I32, I32]),
        "fm_policy_gradient": (I32, [I32, I32, I32, I32, P, P, I32, P, P, I32, I32, ctypes.c_float, U64, I64,
                                     I32, ctypes.c_float, P, P, SZ, P]),
        "fm_policy_gradient_noalloc": (I32, [I32, I32, I32, I32, P, P, I32, P, P, I32, I32, ctypes.c_float, U64,
                                             I64, I32, ctypes.c_float, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != FM_OK:
        raise FmError(status, load().fm_last_error().decode())


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def make_config(cfg) -> FmEnvConfig:
    """FmEnvConfig from any object with the fields of workload.EnvConfig."""
    return FmEnvConfig(cfg.n_envs, cfg.n_stocks, cfg.n_ind, cfg.n_days, cfg.hmax, cfg.init_cash,
                       cfg.cost_rate, cfg.reward_scale, cfg.cash_obs_scale, cfg.price_obs_scale,
                       cfg.hold_obs_scale)


# --- entry points, same names as the C ABI ---------------------------------------------------

def env_workspace_bytes(cfg) -> int:
    c = cfg if isinstance(cfg, FmEnvConfig) else make_config(cfg)
    return int(load().env_workspace_bytes(ctypes.byref(c)))


def env_create(cfg, d_close, d_ind, d_workspace, stream=None):
    import torch
    c = cfg if isinstance(cfg, FmEnvConfig) else make_config(cfg)
    h = ctypes.c_void_p()
    _check(load().env_create(ctypes.byref(c), _ptr(d_close, torch.float32, name="close"),
                             _ptr(d_ind, torch.float32, name="ind"), _ptr(d_workspace, name="workspace"),
                             d_workspace.numel() * d_workspace.element_size(), _stream(stream),
                             ctypes.byref(h)))
    return h


def env_reset(env, d_obs=None):
    import torch
    _check(load().env_reset(env, _ptr(d_obs, torch.float32, name="obs")))


def env_step(env, d_act, d_reward, d_obs=None, d_exec_qty=None) -> bool:
    import torch
    done = ctypes.c_int32(0)
    _check(load().env_step(env, _ptr(d_act, torch.float32, name="act"), _ptr(d_obs, torch.float32, name="obs"),
                           _ptr(d_reward, torch.float64, name="reward"),
                           _ptr(d_exec_qty, torch.int32, name="exec_qty"), ctypes.byref(done)))
    return bool(done.value)


def env_rollout(env, ens, n_steps, d_actions=None, sigma=0.0, noise_key=0, env_offset=0, path=FM_PATH_PLAIN,
                d_obs_traj=None, d_act_traj=None, d_rew_traj=None, d_qty_traj=None):
    import torch
    o = FmRolloutOpts(_ptr(d_actions, torch.float32, name="actions"), float(sigma), int(noise_key),
                      int(env_offset), int(path), _ptr(d_obs_traj, torch.float32, name="obs_traj"),
                      _ptr(d_act_traj, torch.float32, name="act_traj"),
                      _ptr(d_rew_traj, torch.float64, name="rew_traj"),
                      _ptr(d_qty_traj, torch.int32, name="qty_traj"))
    _check(load().env_rollout(env, ens, int(n_steps), ctypes.byref(o)))


def env_read_state(env, d_cash=None, d_hold=None, d_asset=None, d_cumrew=None) -> int:
    import torch
    day = ctypes.c_int32(0)
    _check(load().env_read_state(env, _ptr(d_cash, torch.float64, name="cash"), _ptr(d_hold, torch.int32, name="hold"),
                                 _ptr(d_asset, torch.float64, name="asset"),
                                 _ptr(d_cumrew, torch.float64, name="cumrew"), ctypes.byref(day)))
    return int(day.value)


def env_write_state(env, d_cash, d_hold, d_asset, d_cumrew, day: int):
    import torch
    _check(load().env_write_state(env, _ptr(d_cash, torch.float64, name="cash"), _ptr(d_hold, torch.int32, name="hold"),
                                  _ptr(d_asset, torch.float64, name="asset"),
                                  _ptr(d_cumrew, torch.float64, name="cumrew"), int(day)))


def env_day(env) -> int:
    return int(load().env_day(env))


def env_set_tile(env, envs_per_group: int) -> int:
    out = ctypes.c_int32(0)
    _check(load().env_set_tile(env, int(envs_per_group), ctypes.byref(out)))
    return out.value


def env_set_step_kernel(env, kernel=0, envs_per_wave=0):
    _check(load().env_set_step_kernel(env, int(kernel), int(envs_per_wave)))


def env_set_fused_tuning(env, schedule=0, row_tiles=0, tile_envs=0):
    _check(load().env_set_fused_tuning(env, int(schedule), int(row_tiles), int(tile_envs)))


def env_destroy(env):
    load().env_destroy(env)


def ensemble_workspace_bytes(n_actors, in_dim, hidden, out_dim, dtype, max_batch) -> int:
    return int(load().ensemble_workspace_bytes(n_actors, in_dim, hidden, out_dim, dtype, max_batch))


def ensemble_create(n_actors, in_dim, hidden, out_dim, dtype, d_w, mix, max_batch, d_workspace, stream=None):
    import torch
    h = ctypes.c_void_p()
    mix_arr = None
    if mix is not None:
        mix_arr = (ctypes.c_float * n_actors)(*[float(x) for x in mix])
    _check(load().ensemble_create(n_actors, in_dim, hidden, out_dim, dtype, _ptr(d_w, torch.float32, name="weights"),
                                  mix_arr, max_batch, _ptr(d_workspace, name="workspace"),
                                  d_workspace.numel() * d_workspace.element_size(), _stream(stream),
                                  ctypes.byref(h)))
    return h


def ensemble_act(ens, d_obs, n, sigma, noise_key, t, env_offset, d_act, d_mean=None, stream=None):
    import torch
    _check(load().ensemble_act(ens, _ptr(d_obs, torch.float32, name="obs"), int(n), float(sigma), int(noise_key),
                               int(t), int(env_offset), _ptr(d_mean, torch.float32, name="mean"),
                               _ptr(d_act, torch.float32, name="act"), _stream(stream)))


def ensemble_destroy(ens):
    load().ensemble_destroy(ens)


def fm_noise(noise_key, env_offset, n, t, n_stocks, d_eps, d_words=None, stream=None):
    import torch
    _check(load().fm_noise(int(noise_key), int(env_offset), int(n), int(t), int(n_stocks),
                           _ptr(d_words, torch.int64, name="words"), _ptr(d_eps, torch.float32, name="eps"),
                           _stream(stream)))


METRICS = ("cumulative_return", "annual_return", "annual_volatility", "sharpe", "max_drawdown", "romad",
           "sortino", "calmar", "omega", "win_loss")


def fm_backtest_metrics(d_rew, init_asset, reward_scale, periods_per_year=252.0, risk_free=0.0, d_init_asset=None,
                        d_out=None, stream=None):
    """Metrics [N][10] (order of METRICS) from rewards [T][N] float64 on the device."""
    import torch
    T, N = d_rew.shape
    if d_out is None:
        d_out = torch.empty((N, len(METRICS)), dtype=torch.float64, device=d_rew.device)
    _check(load().fm_backtest_metrics(_ptr(d_rew, torch.float64, name="rew"), int(T), int(N), float(init_asset),
                                      _ptr(d_init_asset, torch.float64, N, name="init_asset"), float(reward_scale),
                                      float(periods_per_year), float(risk_free),
                                      _ptr(d_out, torch.float64, N * len(METRICS), name="out"), _stream(stream)))
    return d_out


def fm_sharpe_weights(sharpe, min_sharpe=float("-inf")):
    """Softmax-of-Sharpe ensemble weights (host)."""
    K = len(sharpe)
    s = (ctypes.c_double * K)(*[float(x) for x in sharpe])
    w = (ctypes.c_float * K)()
    _check(load().fm_sharpe_weights(s, K, float(min_sharpe), w))
    return [float(x) for x in w]


def fm_last_error() -> str:
    return load().fm_last_error().decode()


def fm_version() -> str:
    return load().fm_version().decode()


def make_batch_groups(groups):
    """Array of FmBatchGroup from dicts with keys env (handle), ens (handle), n_steps, sigma,
    noise_key, env_offset and optional obs/act/rew/qty trajectory tensors."""
    import torch
    arr = (FmBatchGroup * len(groups))()
    for i, g in enumerate(groups):
        arr[i] = FmBatchGroup(g["env"], g["ens"], int(g["n_steps"]), float(g.get("sigma", 0.0)),
                              int(g.get("noise_key", 0)), int(g.get("env_offset", 0)),
                              _ptr(g.get("obs"), torch.float32, name="obs_traj"),
                              _ptr(g.get("act"), torch.float32, name="act_traj"),
                              _ptr(g.get("rew"), torch.float64, name="rew_traj"),
                              _ptr(g.get("qty"), torch.int32, name="qty_traj"))
    return arr


def fm_batch_workspace_bytes(groups) -> int:
    arr = groups if isinstance(groups, ctypes.Array) else make_batch_groups(groups)
    return int(load().fm_batch_workspace_bytes(arr, len(arr)))


def fm_batch_create(groups, d_workspace, stream=None):
    arr = groups if isinstance(groups, ctypes.Array) else make_batch_groups(groups)
    h = ctypes.c_void_p()
    _check(load().fm_batch_create(arr, len(arr), _ptr(d_workspace, name="workspace"),
                                  d_workspace.numel() * d_workspace.element_size(), _stream(stream), ctypes.byref(h)))
    return h


def fm_batch_tune(batch):
    rows, blocks = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().fm_batch_tune(batch, ctypes.byref(rows), ctypes.byref(blocks)))
    return rows.value, blocks.value


def fm_batch_set_tiling(batch, rows, blocks):
    _check(load().fm_batch_set_tiling(batch, int(rows), int(blocks)))


def fm_batch_run(batch, use_graph=False):
    _check(load().fm_batch_run(batch, 1 if use_graph else 0))


def fm_batch_destroy(batch):
    load().fm_batch_destroy(batch)



# ------------------------------------------------------------------------------------------------
# Crypto serving (include/crypto_serve.h)
# ------------------------------------------------------------------------------------------------

def fm_serve_request_bytes(n_envs: int) -> int:
    return int(load().fm_serve_request_bytes(int(n_envs)))


def fm_serve_workspace_bytes(cfg: FmServeConfig) -> int:
    return int(load().fm_serve_workspace_bytes(ctypes.byref(cfg)))


def fm_serve_create(cfg: FmServeConfig, stream=None):
    out = ctypes.c_void_p()
    _check(load().fm_serve_create(ctypes.byref(cfg), _stream(stream), ctypes.byref(out)))
    return out


def fm_serve_submit(server, req: FmServeRequest) -> int:
    rid = ctypes.c_int64()
    _check(load().fm_serve_submit(server, ctypes.byref(req), ctypes.byref(rid)))
    return rid.value


def fm_serve_step(server, stream=None):
    """(active requests, queued requests) after the step."""
    a, q = ctypes.c_int32(), ctypes.c_int32()
    _check(load().fm_serve_step(server, _stream(stream), ctypes.byref(a), ctypes.byref(q)))
    return a.value, q.value


def fm_serve_poll(server, wait=False, cap=4096):
    ids = (ctypes.c_int64 * cap)()
    n = ctypes.c_int32()
    _check(load().fm_serve_poll(server, 1 if wait else 0, ids, cap, ctypes.byref(n)))
    return [ids[i] for i in range(n.value)]


def fm_serve_destroy(server):
    load().fm_serve_destroy(server)


# ------------------------------------------------------------------------------------------------
# Learner (include/learner.h)
# ------------------------------------------------------------------------------------------------

def fm_pg_workspace_bytes(K, S, H, A, N, T) -> int:
    return int(load().fm_pg_workspace_bytes(K, S, H, A, N, T))


def fm_policy_gradient(K, S, H, A, d_w, agent, d_states, d_rew, N, T, sigma, noise_key, env_offset, lambda_kl,
                       d_grad, d_workspace, mix=None, stream=None, t0=0):
    """Gradient of agent `agent`'s objective (eqs. 4 and 5) into d_grad (float32, one actor's
    master-weight layout).  t0: the day of the first sample row."""
    import numpy as np
    import torch
    h_mix = None
    if mix is not None:
        h_mix = np.ascontiguousarray(mix, dtype=np.float32)
    per = S * H + H + H * H + H + H * A + A
    _check(load().fm_policy_gradient(
        K, S, H, A, _ptr(d_w, torch.float32, K * per, "d_w"), None if h_mix is None else h_mix.ctypes.data, agent,
        _ptr(d_states, torch.float32, T * N * S, "d_states"), _ptr(d_rew, torch.float64, T * N, "d_rew"), N, T,
        float(sigma), int(noise_key), int(env_offset), int(t0), float(lambda_kl),
        _ptr(d_grad, torch.float32, per, "d_grad"),
        _ptr(d_workspace, None, None, "d_workspace"), d_workspace.numel() * d_workspace.element_size(),
        _stream(stream)))


def fm_policy_gradient_noalloc(K, S, H, A, d_w, agent, d_states, d_rew, N, T, sigma, noise_key, env_offset, lambda_kl,
                               d_grad, mix=None, stream=None, t0=0):
    """fm_policy_gradient with the library's own device scratch instead of a workspace argument
    (for callers that cannot allocate; at most FM_PG_NOALLOC_MAX_BYTES of workspace)."""
    import numpy as np
    import torch
    h_mix = None
    if mix is not None:
        h_mix = np.ascontiguousarray(mix, dtype=np.float32)
    per = S * H + H + H * H + H + H * A + A
    _check(load().fm_policy_gradient_noalloc(
        K, S, H, A, _ptr(d_w, torch.float32, K * per, "d_w"), None if h_mix is None else h_mix.ctypes.data, agent,
        _ptr(d_states, torch.float32, T * N * S, "d_states"), _ptr(d_rew, torch.float64, T * N, "d_rew"), N, T,
        float(sigma), int(noise_key), int(env_offset), int(t0), float(lambda_kl),
        _ptr(d_grad, torch.float32, per, "d_grad"), _stream(stream)))
