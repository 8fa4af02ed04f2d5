"""The learner on the GPU (include/learner.h) against the oracle: the policy gradient of eq. (4)
with the KL diversity term of eq. (5), computed from a real rollout's stored states and rewards.

Tolerance: float32 forward and backward passes (fixed summation orders) against float64; every
entry within 1e-5 of the largest entry of that parameter's gradient (the observed error is about
1e-7 of it), plus the bit-identical repeat of a call."""
import numpy as np
import pytest

from oracle import learner as OL
from workload import ActorConfig, EnvConfig, make_actor_weights, make_market, pack_actor_weights

pytestmark = pytest.mark.gpu
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def _rollout(N, D, T, K, H, sigma, key, env_offset, seed, t0=0):
    """T sampled steps from day t0: the first t0 steps run as a separate rollout whose samples are
    dropped, so the kept samples come from a rollout resumed on day t0."""
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    cfg = EnvConfig(n_envs=N, n_stocks=D, n_ind=5, n_days=t0 + T)
    m = make_market(seed, D, t0 + T)
    acfg = ActorConfig(n_actors=K, in_dim=cfg.state_dim, hidden=H, out_dim=D, bias_std=0.1, seed_base=300 + seed)
    actors = make_actor_weights(acfg)
    env = VecEnv(cfg, m.close, m.ind, device=torch.device("cuda:0"))
    ens = Ensemble(pack_actor_weights(actors), K, cfg.state_dim, H, D, dtype="f32", max_batch=N)
    s0 = env.reset()
    if t0 > 0:
        first = env.rollout(t0, ens=ens, sigma=sigma, noise_key=key, env_offset=env_offset, path="plain",
                            store=("obs",))
        s0 = first["obs"][-1]
        assert env.day == t0
    out = env.rollout(T, ens=ens, sigma=sigma, noise_key=key, env_offset=env_offset, path="plain", store=("obs", "rew"))
    states = torch.cat([s0[None], out["obs"][:-1]], 0).contiguous()
    return cfg, actors, states, out["rew"].contiguous()


def _unflatten(flat, S, H, A):
    out, o = {}, 0
    for name, shp in (("W1", (S, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, A)), ("b3", (A,))):
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    return out


@pytest.mark.parametrize("agent,lam,N,T,K,H,t0", [(0, 0.0, 24, 16, 3, 64, 0), (2, 0.5, 37, 9, 3, 64, 0),
                                                  (1, 2.0, 130, 5, 3, 64, 0), (0, 1.0, 1, 1, 1, 64, 0),
                                                  (1, 0.3, 50, 7, 3, 128, 0), (2, 0.4, 40, 6, 3, 64, 5)])
def test_policy_gradient_matches_oracle(agent, lam, N, T, K, H, t0):
    """The fourth case is degenerate: one actor (no diversity term whatever lambda), one
    environment, one day.  The fifth has a hidden width of one row tile (128), where the bias
    gradients come from column sums inside the weight-gradient product.  The last takes its
    samples from a rollout resumed on day 5: the regenerated noise must be that of days 5..10."""
    import torch
    from paper_2501_10709_amd import binding as B
    D, sigma, key, off = 5, 0.1, 9, 4
    cfg, actors, states, rew = _rollout(N, D, T, K, H, sigma, key, off, seed=agent + 3, t0=t0)
    S, A = cfg.state_dim, D
    w = torch.as_tensor(pack_actor_weights(actors)).cuda()
    per = S * H + H + H * H + H + H * A + A
    ws = torch.empty(B.fm_pg_workspace_bytes(K, S, H, A, N, T), dtype=torch.uint8, device="cuda")
    g1 = torch.empty(per, dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    print(f"policy gradient agent {agent} lambda {lam} N {N} T {T} K {K} H {H} t0 {t0}", flush=True)
    B.fm_policy_gradient(K, S, H, A, w, agent, states, rew, N, T, sigma, key, off, lam, g1, ws, t0=t0)
    B.fm_policy_gradient(K, S, H, A, w, agent, states, rew, N, T, sigma, key, off, lam, g2, ws, t0=t0)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    got = _unflatten(g1.cpu().numpy().astype(np.float64), S, H, A)
    want = OL.policy_gradient(actors, agent, states.cpu().numpy(), rew.cpu().numpy(), sigma, key, off, lam, t0=t0)
    for name in NAMES:
        scale = np.abs(want[name]).max()
        assert scale > 0, name
        err = np.abs(got[name] - want[name]).max()
        print(f"  {name}: max error {err / scale:.2e} of scale", flush=True)
        assert err <= 1e-5 * scale, (name, err, scale)
    if t0 > 0:
        # Keyed by the row index instead of the day, the layer-3 gradient would differ.
        wrong = OL.policy_gradient(actors, agent, states.cpu().numpy(), rew.cpu().numpy(), sigma, key, off, lam)
        assert np.abs(wrong["b3"] - got["b3"]).max() > 1e-3 * np.abs(want["b3"]).max()


def test_policy_gradient_argument_errors():
    import torch
    from paper_2501_10709_amd import binding as B
    K, S, H, A, N, T = 2, 8, 16, 3, 4, 2
    w = torch.zeros(K * (S * H + H + H * H + H + H * A + A), device="cuda")
    st = torch.zeros((T, N, S), device="cuda")
    rw = torch.zeros((T, N), dtype=torch.float64, device="cuda")
    g = torch.zeros(S * H + H + H * H + H + H * A + A, device="cuda")
    ws = torch.empty(B.fm_pg_workspace_bytes(K, S, H, A, N, T), dtype=torch.uint8, device="cuda")
    for kw in (dict(agent=2), dict(sigma=0.0), dict(lam=-1.0), dict(t0=-1)):
        with pytest.raises(B.FmError):
            B.fm_policy_gradient(K, S, H, A, w, kw.get("agent", 0), st, rw, N, T, kw.get("sigma", 0.1), 1, 0,
                                 kw.get("lam", 0.0), g, ws, t0=kw.get("t0", 0))
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.FmError):
        B.fm_policy_gradient(K, S, H, A, w, 0, st, rw, N, T, 0.1, 1, 0, 0.0, g, small)
