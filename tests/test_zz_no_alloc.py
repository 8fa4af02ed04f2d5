"""The allocation-free learner entry point (fm_policy_gradient_noalloc, include/learner.h) against
fm_policy_gradient with a caller workspace: two calls in a row on the same device, the second
smaller than the first, each bit-identical to the workspace entry point on the same inputs (both
run the same kernels in the same order).  A problem larger than the library's scratch is rejected
before anything is enqueued."""
import numpy as np
import pytest

from workload import ActorConfig, EnvConfig, make_actor_weights, make_market, pack_actor_weights

pytestmark = pytest.mark.gpu


def _samples(N, D, T, K, H, seed):
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    cfg = EnvConfig(n_envs=N, n_stocks=D, n_ind=5, n_days=T)
    m = make_market(seed, D, T)
    acfg = ActorConfig(n_actors=K, in_dim=cfg.state_dim, hidden=H, out_dim=D, bias_std=0.1, seed_base=500 + seed)
    packed = pack_actor_weights(make_actor_weights(acfg))
    env = VecEnv(cfg, m.close, m.ind, device=torch.device("cuda:0"))
    ens = Ensemble(packed, K, cfg.state_dim, H, D, dtype="f32", max_batch=N)
    s0 = env.reset()
    out = env.rollout(T, ens=ens, sigma=0.1, noise_key=11, path="plain", store=("obs", "rew"))
    states = torch.cat([s0[None], out["obs"][:-1]], 0).contiguous()
    return cfg.state_dim, torch.as_tensor(packed).cuda(), states, out["rew"].contiguous()


@pytest.mark.parametrize("first,second", [((96, 30, 30, 3, 64, 1, 0.5), (17, 7, 30, 3, 64, 2, 0.1)),
                                          ((40, 12, 30, 3, 256, 0, 1.0), (5, 3, 30, 3, 256, 2, 0.0))])
def test_noalloc_matches_workspace_entry_point(first, second):
    import torch
    from paper_2501_10709_amd import binding as B
    for N, T, D, K, H, agent, lam in (first, second):
        S, w, states, rew = _samples(N, D, T, K, H, seed=N)
        assert B.fm_pg_workspace_bytes(K, S, H, D, N, T) <= 32 << 20
        per = S * H + H + H * H + H + H * D + D
        g_ws = torch.empty(per, dtype=torch.float32, device="cuda")
        g_na = torch.full((per,), float("nan"), dtype=torch.float32, device="cuda")
        ws = torch.empty(B.fm_pg_workspace_bytes(K, S, H, D, N, T), dtype=torch.uint8, device="cuda")
        print(f"noalloc N {N} T {T} H {H} agent {agent} lambda {lam}", flush=True)
        B.fm_policy_gradient(K, S, H, D, w, agent, states, rew, N, T, 0.1, 11, 0, lam, g_ws, ws, t0=0)
        B.fm_policy_gradient_noalloc(K, S, H, D, w, agent, states, rew, N, T, 0.1, 11, 0, lam, g_na, t0=0)
        torch.cuda.synchronize()
        assert torch.isfinite(g_na).all()
        assert torch.equal(g_ws, g_na)


def test_noalloc_rejects_problems_beyond_its_scratch():
    import torch
    from paper_2501_10709_amd import binding as B
    K, S, H, A, N, T = 3, 211, 256, 30, 256, 64
    assert B.fm_pg_workspace_bytes(K, S, H, A, N, T) > 32 << 20
    per = S * H + H + H * H + H + H * A + A
    w = torch.zeros(K * per, device="cuda")
    st = torch.zeros((T, N, S), device="cuda")
    rw = torch.zeros((T, N), dtype=torch.float64, device="cuda")
    g = torch.zeros(per, device="cuda")
    with pytest.raises(B.FmError, match="more than"):
        B.fm_policy_gradient_noalloc(K, S, H, A, w, 0, st, rw, N, T, 0.1, 1, 0, 0.0, g)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(g)) == 0
