"""The C ABI without a GPU: the library loads, exports every declared symbol, and the host-side
validation rejects bad arguments before anything reaches the device."""
import ctypes
import os
import re

import numpy as np

import pytest

from paper_2501_10709_amd import binding as B
from workload import PAPER_SCALE, TINY

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text,
                            flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_version(lib):
    assert "gfx950" in B.fm_version()


def test_env_workspace_bytes():
    n = B.env_workspace_bytes(PAPER_SCALE.env)
    N, D, S = 2048, 30, 211
    assert n >= 3 * 8 * N + 4 * D * N + 4 * D * N + 4 * S * N
    assert n % 256 == 0
    for bad in (dict(n_envs=0), dict(n_stocks=0), dict(n_stocks=129), dict(n_ind=17), dict(n_days=0),
                dict(hmax=0), dict(cost_rate=1.0), dict(cost_rate=-0.1), dict(init_cash=-1.0),
                dict(init_cash=float("inf")), dict(reward_scale=float("nan"))):
        assert B.env_workspace_bytes(TINY.env.replace(**bad)) == 0, bad


def test_ensemble_workspace_bytes():
    ok = B.ensemble_workspace_bytes(3, 211, 256, 30, B.FM_BF16, 2048)
    weights_bf16 = 3 * 2 * (224 * 256 + 256 * 256 + 256 * 32)
    mu = 3 * 2048 * 30 * 4
    assert ok >= weights_bf16 + mu
    assert B.ensemble_workspace_bytes(3, 211, 256, 30, B.FM_F32, 2048) > ok
    for bad in ((0, 211, 256, 30, 0, 1), (9, 211, 256, 30, 0, 1), (3, 211, 250, 30, 0, 1),
                (3, 211, 1024, 30, 0, 1), (3, 0, 256, 30, 0, 1), (3, 211, 256, 129, 0, 1),
                (3, 211, 256, 30, 2, 1), (3, 211, 256, 30, 0, 0)):
        assert B.ensemble_workspace_bytes(*bad) == 0, bad


def test_invalid_arguments_return_error_without_device(lib):
    cfg = B.make_config(TINY.env)
    h = ctypes.c_void_p()
    # NULL market pointer: rejected before any device call.
    st = lib.env_create(ctypes.byref(cfg), None, None, None, 0, None, ctypes.byref(h))
    assert st == B.FM_ERR_INVALID and "NULL" in B.fm_last_error()
    bad = B.make_config(TINY.env.replace(n_stocks=500))
    st = lib.env_create(ctypes.byref(bad), ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                        1 << 30, None, ctypes.byref(h))
    assert st == B.FM_ERR_INVALID and "n_stocks" in B.fm_last_error()
    # Misaligned workspace.
    st = lib.env_create(ctypes.byref(cfg), ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(1028),
                        1 << 30, None, ctypes.byref(h))
    assert st == B.FM_ERR_INVALID and "aligned" in B.fm_last_error()
    # Too small a workspace.
    st = lib.env_create(ctypes.byref(cfg), ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                        16, None, ctypes.byref(h))
    assert st == B.FM_ERR_INVALID and "small" in B.fm_last_error()
    # NULL handles.
    assert lib.env_reset(None, None) == B.FM_ERR_INVALID
    assert lib.env_step(None, None, None, None, None, None) == B.FM_ERR_INVALID
    assert lib.env_rollout(None, None, 1, None) == B.FM_ERR_INVALID
    assert lib.ensemble_act(None, None, 1, 0.0, 0, 0, 0, None, None, None) == B.FM_ERR_INVALID
    assert lib.env_day(None) == -1
    # Ensemble argument checks.
    e = ctypes.c_void_p()
    assert lib.ensemble_create(3, 211, 100, 30, 0, ctypes.c_void_p(256), None, 16, ctypes.c_void_p(1024), 1 << 30,
                               None, ctypes.byref(e)) == B.FM_ERR_INVALID
    assert "hidden" in B.fm_last_error()
    assert lib.fm_noise(7, 0, 4, 0, 30, None, None, None) == B.FM_ERR_INVALID


def test_sharpe_weights_match_oracle():
    from oracle.metrics import sharpe_softmax_weights
    for s, cut in (([0.7, 0.7, 0.7], float("-inf")), ([1.0, 2.0, 0.5], float("-inf")), ([1.0, -0.5, 2.0], 0.0),
                   ([-1.0, -0.2, -3.0], 0.0), ([3.0], 0.0), ([0.1, 0.4, 0.2, 0.9, -2.0], 0.15)):
        got = np.array(B.fm_sharpe_weights(s, cut))
        want = sharpe_softmax_weights(s, cut)
        assert np.allclose(got, want, rtol=1e-6, atol=1e-7), (s, got, want)
    with pytest.raises(B.FmError):
        B.fm_sharpe_weights([float("nan"), 1.0])


def test_env_set_tile_validation(lib):
    assert lib.env_set_tile(None, 8, None) == B.FM_ERR_INVALID
    assert "NULL" in B.fm_last_error()
    assert lib.env_set_fused_tuning(None, 0, 0, 0) == B.FM_ERR_INVALID
    assert "NULL" in B.fm_last_error()
    assert lib.env_set_step_kernel(None, 0, 0) == B.FM_ERR_INVALID
    assert "NULL" in B.fm_last_error()


def test_batch_argument_validation(lib):
    assert lib.fm_batch_workspace_bytes(None, 0) == 0
    h = ctypes.c_void_p()
    assert lib.fm_batch_create(None, 1, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h)) == B.FM_ERR_INVALID
    assert "NULL" in B.fm_last_error()
    groups = (B.FmBatchGroup * 1)()
    assert lib.fm_batch_workspace_bytes(groups, 1) == 0  # NULL env / ensemble
    assert lib.fm_batch_run(None, 0) == B.FM_ERR_INVALID
    assert lib.fm_batch_tune(None, None, None) == B.FM_ERR_INVALID
    assert lib.fm_batch_set_tiling(None, 16, 256) == B.FM_ERR_INVALID


def test_serve_config_validation(lib):
    cfg = B.FmServeConfig()
    assert B.fm_serve_workspace_bytes(cfg) == 0          # NULL tick table
    w = np.zeros(5 * (16 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3), np.float32)
    cfg.d_mid, cfg.d_feat, cfg.n_ticks = 256, 256, 1000
    cfg.n_agents, cfg.h_weights, cfg.rule, cfg.eps, cfg.fee, cfg.cash0 = 5, w.ctypes.data, 0, 0.0, 2e-4, 1e5
    cfg.tile_rows, cfg.chunk_ticks, cfg.max_requests, cfg.max_active_envs = 64, 256, 16, 4096
    cfg.d_pool, cfg.pool_bytes = 256, 1 << 20
    n = B.fm_serve_workspace_bytes(cfg)
    assert n > 5 * 32 * 1024
    for field, bad in [("tile_rows", 32), ("n_agents", 4), ("eps", 1.5), ("chunk_ticks", 0), ("rule", 7)]:
        old = getattr(cfg, field)
        setattr(cfg, field, bad)
        assert B.fm_serve_workspace_bytes(cfg) == 0, field
        out = ctypes.c_void_p()
        assert lib.fm_serve_create(ctypes.byref(cfg), None, ctypes.byref(out)) == B.FM_ERR_INVALID
        assert not out.value and B.fm_last_error()
        setattr(cfg, field, old)
    assert B.fm_serve_request_bytes(0) == 0 and B.fm_serve_request_bytes(1) == 256
    assert B.fm_serve_request_bytes(100) == 6400


def test_pg_workspace_validation(lib):
    assert B.fm_pg_workspace_bytes(3, 211, 256, 30, 2048, 252) > 0
    for bad in ((0, 211, 256, 30, 2048, 252), (9, 211, 256, 30, 2048, 252), (3, 211, 256, 200, 2048, 252),
                (3, 211, 256, 30, 0, 252), (3, 211, 2048, 30, 16, 4)):
        assert B.fm_pg_workspace_bytes(*bad) == 0, bad
