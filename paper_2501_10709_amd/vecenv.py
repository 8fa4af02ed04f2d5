"""Owning wrappers over the C ABI: device buffers come from torch, compute from the library.

VecEnv is the paper's vectorised environment (Section 4.2) over one market; Ensemble is the
K-actor stock ensemble (Section 5.2.1).  Both only allocate torch tensors and call the binding.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def _dev(device):
    return torch.device(device if device is not None else "cuda")


class Ensemble:
    """K actors S -> H -> H -> A packed for the device (float32 or bfloat16 MFMA)."""

    def __init__(self, packed_weights, n_actors, in_dim, hidden, out_dim, dtype="f32", max_batch=1,
                 mix=None, device=None):
        dev = _dev(device)
        self.K, self.S, self.H, self.A = int(n_actors), int(in_dim), int(hidden), int(out_dim)
        self.dtype = {"f32": B.FM_F32, "bf16": B.FM_BF16}[dtype]
        self.dtype_name = dtype
        self.max_batch = int(max_batch)
        w = torch.as_tensor(np.ascontiguousarray(packed_weights, dtype=np.float32)).to(dev)
        nbytes = B.ensemble_workspace_bytes(self.K, self.S, self.H, self.A, self.dtype, self.max_batch)
        if nbytes == 0:
            raise ValueError("unsupported ensemble shape")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.handle = B.ensemble_create(self.K, self.S, self.H, self.A, self.dtype, w, mix, self.max_batch,
                                        self.workspace)
        self.device = dev

    def act(self, obs, t, sigma=0.0, noise_key=0, env_offset=0, return_mean=False):
        obs = obs.contiguous()
        if obs.dim() != 2 or obs.shape[1] != self.S or obs.shape[0] > self.max_batch:
            raise ValueError(f"obs must be [n <= {self.max_batch}][{self.S}], got {tuple(obs.shape)}")
        n = obs.shape[0]
        act = torch.empty((n, self.A), dtype=torch.float32, device=self.device)
        mean = torch.empty_like(act) if return_mean else None
        B.ensemble_act(self.handle, obs, n, sigma, noise_key, t, env_offset, act, mean)
        return (act, mean) if return_mean else act

    def close(self):
        if self.handle is not None:
            B.ensemble_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VecEnv:
    """N sub-environments on one market path: reset / step / reward and T-step rollouts."""

    def __init__(self, cfg, close, ind, device=None):
        dev = _dev(device)
        self.cfg = cfg
        self.N, self.D, self.I, self.T = cfg.n_envs, cfg.n_stocks, cfg.n_ind, cfg.n_days
        self.S = (self.I + 2) * self.D + 1
        self.close = torch.as_tensor(np.ascontiguousarray(close, dtype=np.float32)).to(dev)
        self.ind = torch.as_tensor(np.ascontiguousarray(ind, dtype=np.float32)).to(dev)
        if tuple(self.close.shape) != (self.T + 1, self.D) or tuple(self.ind.shape) != (self.T + 1, self.I, self.D):
            raise ValueError("market arrays do not match the configuration")
        nbytes = B.env_workspace_bytes(cfg)
        if nbytes == 0:
            raise ValueError("invalid environment configuration")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.handle = B.env_create(cfg, self.close, self.ind, self.workspace)
        self.device = dev

    @property
    def day(self) -> int:
        return B.env_day(self.handle)

    def set_tile(self, envs_per_group: int) -> int:
        """Environments per workgroup of the environment kernels (0: size-based default)."""
        return B.env_set_tile(self.handle, envs_per_group)

    def set_step_kernel(self, kernel=0, envs_per_wave=0):
        """Environment-step kernel: 0 by shape and size, 1 the tile kernel, 2 one lane per
        environment, 3 a 16-lane row per environment; environments per wavefront of the lane
        kernel (0: by N)."""
        B.env_set_step_kernel(self.handle, kernel, envs_per_wave)

    def set_fused_tuning(self, schedule=0, row_tiles=0, tile_envs=0):
        """Fused-rollout tuning: schedule (0 by shape and size, 1 streamed, 2 generic, 3 resident),
        MFMA row tiles per workgroup (1, 2; 0 by N) and environments per workgroup (0: fill the
        compute units)."""
        B.env_set_fused_tuning(self.handle, schedule, row_tiles, tile_envs)

    def reset(self, return_obs=True):
        obs = torch.empty((self.N, self.S), dtype=torch.float32, device=self.device) if return_obs else None
        B.env_reset(self.handle, obs)
        return obs

    def step(self, act, return_obs=True, return_qty=True):
        act = act.contiguous()
        if tuple(act.shape) != (self.N, self.D):
            raise ValueError(f"act must have shape {(self.N, self.D)}, got {tuple(act.shape)}")
        rew = torch.empty(self.N, dtype=torch.float64, device=self.device)
        obs = torch.empty((self.N, self.S), dtype=torch.float32, device=self.device) if return_obs else None
        qty = torch.empty((self.N, self.D), dtype=torch.int32, device=self.device) if return_qty else None
        done = B.env_step(self.handle, act, rew, obs, qty)
        return obs, rew, qty, done

    def rollout(self, n_steps, ens=None, actions=None, sigma=0.0, noise_key=0, env_offset=0, path="plain",
                store=("obs", "act", "rew", "qty"), out=None):
        """Run n_steps steps; returns dict of [n_steps][N][...] trajectories for the names in store.

        out: optional dict of preallocated trajectory tensors (reused across calls).
        """
        p = {"plain": B.FM_PATH_PLAIN, "fused": B.FM_PATH_FUSED}[path]
        T, N, D, S = n_steps, self.N, self.D, self.S
        if actions is not None and tuple(actions.shape) != (T, N, D):
            raise ValueError(f"actions must have shape {(T, N, D)}, got {tuple(actions.shape)}")
        shapes = {"obs": ((T, N, S), torch.float32), "act": ((T, N, D), torch.float32),
                  "rew": ((T, N), torch.float64), "qty": ((T, N, D), torch.int32)}
        res = {}
        for k in store:
            if out is not None and k in out:
                if tuple(out[k].shape) != shapes[k][0] or out[k].dtype != shapes[k][1]:
                    raise ValueError(f"out[{k!r}] must be {shapes[k]}")
                res[k] = out[k]
            else:
                shp, dt = shapes[k]
                res[k] = torch.empty(shp, dtype=dt, device=self.device)
        B.env_rollout(self.handle, None if ens is None else ens.handle, n_steps,
                      d_actions=None if actions is None else actions.contiguous(), sigma=sigma, noise_key=noise_key,
                      env_offset=env_offset, path=p, d_obs_traj=res.get("obs"), d_act_traj=res.get("act"),
                      d_rew_traj=res.get("rew"), d_qty_traj=res.get("qty"))
        return res

    def read_state(self):
        d = self.device
        cash = torch.empty(self.N, dtype=torch.float64, device=d)
        asset = torch.empty_like(cash)
        cumrew = torch.empty_like(cash)
        hold = torch.empty((self.N, self.D), dtype=torch.int32, device=d)
        day = B.env_read_state(self.handle, cash, hold, asset, cumrew)
        return dict(cash=cash, hold=hold, asset=asset, cumrew=cumrew, day=day)

    def write_state(self, st):
        d = self.device
        t = lambda x, dt: torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x).to(d, dt).contiguous()
        B.env_write_state(self.handle, t(st["cash"], torch.float64), t(st["hold"], torch.int32),
                          t(st["asset"], torch.float64), t(st["cumrew"], torch.float64), int(st["day"]))

    def close_env(self):
        if self.handle is not None:
            B.env_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close_env()
        except Exception:
            pass


class Batch:
    """Uneven groups of environments stepped together by the batched persistent kernel.

    groups: list of dicts with env (VecEnv), ens (bfloat16 Ensemble), n_steps, and optional
    sigma, noise_key, env_offset, store (names among obs, act, rew, qty; default ("rew",)).
    The trajectories are allocated here: self.out[g][name] is [n_steps][N][...].
    """

    def __init__(self, groups, stream=None):
        dev = groups[0]["env"].device
        self.groups = groups
        self.out = []
        spec = []
        for g in groups:
            env, T = g["env"], int(g["n_steps"])
            shapes = {"obs": ((T, env.N, env.S), torch.float32), "act": ((T, env.N, env.D), torch.float32),
                      "rew": ((T, env.N), torch.float64), "qty": ((T, env.N, env.D), torch.int32)}
            res = {k: torch.empty(shapes[k][0], dtype=shapes[k][1], device=dev) for k in g.get("store", ("rew",))}
            self.out.append(res)
            spec.append(dict(env=env.handle, ens=g["ens"].handle, n_steps=T, sigma=g.get("sigma", 0.0),
                             noise_key=g.get("noise_key", 0), env_offset=g.get("env_offset", 0), **res))
        self._arr = B.make_batch_groups(spec)
        nbytes = B.fm_batch_workspace_bytes(self._arr)
        if nbytes == 0:
            raise ValueError("invalid batch groups")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.handle = B.fm_batch_create(self._arr, self.workspace, stream)

    def tune(self):
        """Autotune the tile rows and persistent grid; returns (rows, blocks)."""
        return B.fm_batch_tune(self.handle)

    def set_tiling(self, rows, blocks):
        """Tile rows (16 or 32) and persistent grid chosen by hand instead of by the autotuner."""
        B.fm_batch_set_tiling(self.handle, rows, blocks)

    def run(self, use_graph=False):
        B.fm_batch_run(self.handle, use_graph)
        return self.out

    def close(self):
        if getattr(self, "handle", None) is not None:
            B.fm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

