"""Owning helper around the crypto serving ABI (include/crypto_serve.h) and a Poisson-arrival
serving loop that measures request latency.

CryptoServer holds the device tick table, pool and workspace (torch tensors) and the per-request
result buffers; every step of the work runs in the library (scheduler in C++, kernels in HIP).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import binding as B

RESULT_DTYPE = np.dtype([("cash", "<f8"), ("value", "<f8"), ("sum_r", "<f8"), ("sum_r2", "<f8"), ("peak", "<f8"),
                         ("max_drawdown", "<f8"), ("position", "<i4"), ("trades", "<i4"), ("ticks", "<i8")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(B.FmCryptoResult) == 64


class CryptoServer:
    def __init__(self, mid, feat, weights, n_agents, rule=B.FM_RULE_AVG_SOFTMAX, eps=0.0, fee=2e-4, cash0=1e5,
                 mix=None, tile_rows=64, chunk_ticks=256, max_requests=4096, max_active_envs=1 << 20,
                 pool_bytes=None, grid=0, device=None, stream=None):
        import torch
        dev = torch.device("cuda:0") if device is None else torch.device(device)
        self.dev = dev
        self.stream = stream
        self.mid = torch.as_tensor(np.ascontiguousarray(mid, np.float64)).to(dev)
        self.feat = torch.as_tensor(np.ascontiguousarray(feat, np.float32)).to(dev)
        if self.feat.ndim != 2 or self.feat.shape[1] != 16 or self.feat.shape[0] != self.mid.shape[0]:
            raise ValueError("feat must be [n_ticks][16] with n_ticks = len(mid)")
        self._weights = np.ascontiguousarray(weights, np.float32)
        self._mix = None if mix is None else np.ascontiguousarray(mix, np.float32)
        if pool_bytes is None:
            pool_bytes = B.fm_serve_request_bytes(1) * max_active_envs
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        cfg = B.FmServeConfig()
        cfg.device = dev.index or 0
        cfg.d_mid = self.mid.data_ptr()
        cfg.d_feat = self.feat.data_ptr()
        cfg.n_ticks = int(self.mid.shape[0])
        cfg.n_agents = int(n_agents)
        cfg.h_weights = self._weights.ctypes.data
        cfg.h_mix = None if self._mix is None else self._mix.ctypes.data
        cfg.rule, cfg.eps, cfg.fee, cfg.cash0 = int(rule), float(eps), float(fee), float(cash0)
        cfg.tile_rows, cfg.chunk_ticks, cfg.max_requests = int(tile_rows), int(chunk_ticks), int(max_requests)
        cfg.max_active_envs, cfg.grid = int(max_active_envs), int(grid)
        cfg.d_pool, cfg.pool_bytes = self.pool.data_ptr(), int(pool_bytes)
        nbytes = B.fm_serve_workspace_bytes(cfg)
        if nbytes == 0:
            raise ValueError("invalid serving configuration: " + B.fm_last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        cfg.d_workspace, cfg.workspace_bytes = self.workspace.data_ptr(), nbytes
        self.cfg = cfg
        self.handle = B.fm_serve_create(cfg, stream)
        self.requests = {}

    def submit(self, n_envs, horizon, start_tick, stride, key, store_act=False, store_prob=False) -> int:
        import torch
        res = torch.empty((n_envs, 64), dtype=torch.uint8, device=self.dev)
        act = torch.empty((horizon, n_envs), dtype=torch.int8, device=self.dev) if store_act else None
        prob = torch.empty((horizon, n_envs, 3), dtype=torch.float32, device=self.dev) if store_prob else None
        r = B.FmServeRequest(n_envs=int(n_envs), stride=int(stride), horizon=int(horizon), start_tick=int(start_tick),
                             key=int(key), d_result=res.data_ptr(),
                             d_act=None if act is None else act.data_ptr(),
                             d_prob=None if prob is None else prob.data_ptr())
        rid = B.fm_serve_submit(self.handle, r)
        self.requests[rid] = (res, act, prob)
        return rid

    def step(self):
        return B.fm_serve_step(self.handle, self.stream)

    def poll(self, wait=False):
        return B.fm_serve_poll(self.handle, wait)

    def result(self, rid, release=True):
        """Per-environment results (structured numpy array) and the stored actions/probabilities."""
        res, act, prob = self.requests.pop(rid) if release else self.requests[rid]
        out = res.cpu().numpy().view(RESULT_DTYPE).reshape(-1)
        return out, (None if act is None else act.cpu().numpy()), (None if prob is None else prob.cpu().numpy())

    def run_all(self):
        """Steps until every submitted request has finished; returns their ids in completion order."""
        done = []
        while True:
            active, queued = self.step()
            done += self.poll()
            if active == 0 and queued == 0:
                done += self.poll(wait=True)
                return done

    def close(self):
        if self.handle:
            B.fm_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_poisson(server: CryptoServer, requests, time_scale: float = 1.0):
    """Continuous-batching loop: request i is submitted once arrival_s * time_scale seconds have
    passed; the loop steps the server and records completion times as the library reports them.
    Returns (latency seconds per request in input order, makespan seconds, env-steps)."""
    n = len(requests)
    arrival = [q.arrival_s * time_scale for q in requests]
    rid_of = {}
    done_at = {}
    i = 0
    t0 = time.perf_counter()
    while len(done_at) < n:
        now = time.perf_counter() - t0
        while i < n and arrival[i] <= now:
            q = requests[i]
            rid_of[server.submit(q.n_envs, q.horizon, q.start_tick, q.stride, q.key)] = i
            i += 1
        active, queued = server.step()
        ids = server.poll()
        if active == 0 and queued == 0:
            ids += server.poll(wait=True)
        t = time.perf_counter() - t0
        for rid in ids:
            done_at[rid_of[rid]] = t
            server.requests.pop(rid, None)
        if active == 0 and queued == 0 and i < n:
            wait = arrival[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    lat = np.array([done_at[j] - arrival[j] for j in range(n)])
    makespan = max(done_at.values()) - arrival[0]
    steps = sum(q.n_envs * q.horizon for q in requests)
    return lat, makespan, steps
