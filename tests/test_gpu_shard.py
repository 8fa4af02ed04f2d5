"""Sharding by environment (each trajectory is an independent simulation, Section 4.1): a rollout
of N environments split into two shards, each its own VecEnv with env_offset = the global index
of its first environment, reproduces the unsplit rollout bit for bit -- states, actions, rewards
and executed quantities -- on the fused bfloat16 path and on the plain float32 path.  This is the
one-GPU check of the multi-GPU layout, where each GPU runs one shard."""
import pytest

from _helpers import actors_case, cuda
from workload import PAPER_SCALE, make_market

pytestmark = pytest.mark.gpu


def _run(cfg, m, packed, H, dtype, path, n, offset, T, dev):
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    c = cfg.replace(n_envs=n)
    ens = Ensemble(packed, 3, c.state_dim, H, c.n_stocks, dtype=dtype, max_batch=n, device=dev)
    env = VecEnv(c, m.close, m.ind, device=dev)
    env.reset(return_obs=False)
    return env.rollout(T, ens=ens, sigma=0.1, noise_key=7, env_offset=offset, path=path)


@pytest.mark.parametrize("dtype,path", [("bf16", "fused"), ("f32", "plain")])
@pytest.mark.parametrize("split", [256, 200])
def test_two_shards_equal_one_run(dtype, path, split):
    import torch
    dev = cuda()
    w = PAPER_SCALE
    N, T = 512, 70
    cfg = w.env.replace(n_envs=N, n_days=T)
    m = make_market(w.market_seed, cfg.n_stocks, T)
    _, _, packed = actors_case(3, cfg.state_dim, w.actors.hidden, cfg.n_stocks, bias_std=0.1)
    print(f"[shard] {path} {dtype} N={N} split {split}+{N - split} T={T}", flush=True)
    whole = _run(cfg, m, packed, w.actors.hidden, dtype, path, N, 0, T, dev)
    a = _run(cfg, m, packed, w.actors.hidden, dtype, path, split, 0, T, dev)
    b = _run(cfg, m, packed, w.actors.hidden, dtype, path, N - split, split, T, dev)
    torch.cuda.synchronize()
    for k in whole:
        joined = torch.cat([a[k], b[k]], dim=1)
        assert torch.equal(joined, whole[k]), k
