"""GPU ensemble, noise and closed-loop rollouts against the CPU oracle.

* Noise: raw Philox4x64-10 words bit-exact; the float32 normals within the bound of their
  float32 evaluation (see _eps_bound).
* ensemble_act on identical states: float32 within 1e-5 and bfloat16 within 2e-2 of the float64
  oracle (which uses the device's bfloat16-rounded weights for the bfloat16 path).
* Closed-loop rollouts (plain and fused): every executed action is replayed through the oracle
  environment, which must reproduce states, quantities and rewards exactly; every action is
  compared with the oracle ensemble acting on the GPU's own state at that step.
"""
import numpy as np
import pytest

from _helpers import TOL_BF16, TOL_F32, actors_case, check_actions, check_replay, cuda, env_case
from oracle.philox import box_muller, noise_words, uniforms_from_words
from oracle.policy import device_weights, ensemble_mean

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _eps_bound(words):
    """|eps_gpu - eps| bound: float32 log (1 ulp), sqrt and product roundings scale with the
    Box-Muller radius r = sqrt(-2 ln u); sincospi adds 2 ulp.  4e-7 * max(1, r)."""
    u = uniforms_from_words(words)
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    r = np.stack([r01, r01, r23, r23], axis=-1)
    return 4e-7 * np.maximum(1.0, r)


@pytest.mark.parametrize("n,t,D,off", [(64, 5, 30, 0), (7, 251, 30, 2041), (33, 0, 5, 123456789), (3, 9, 100, 1)])
def test_noise_words_exact_and_normals_close(n, t, D, off):
    import torch
    from paper_2501_10709_amd import fm_noise
    dev = cuda()
    G = (D + 3) // 4
    words = torch.empty((n, G, 4), dtype=torch.int64, device=dev)
    eps = torch.empty((n, D), dtype=torch.float32, device=dev)
    fm_noise(7, off, n, t, D, eps, words)
    w = _np(words).view(np.uint64)
    ref_w = noise_words(7, np.arange(off, off + n), t, D)
    assert np.array_equal(w, ref_w)
    u = uniforms_from_words(ref_w)
    z0, z1 = box_muller(u[..., 0], u[..., 1])
    z2, z3 = box_muller(u[..., 2], u[..., 3])
    ref = np.stack([z0, z1, z2, z3], axis=-1).reshape(n, -1)[:, :D]
    bound = _eps_bound(ref_w).reshape(n, -1)[:, :D]
    err = np.abs(_np(eps).astype(np.float64) - ref)
    assert np.all(err <= bound), f"worst {err.max():.3e}"


def _obs_sample(n, seed):
    """Realistic states: an oracle environment after a few random steps."""
    from oracle.env import OracleEnv
    from workload import make_actions
    cfg, m = env_case(n, 30, 5, 6, seed)
    env = OracleEnv(cfg, m.close, m.ind)
    env.reset()
    acts = make_actions(seed + 1, 6, n, 30, buy_bias=0.3)
    for t in range(6):
        obs, *_ = env.step(acts[t])
    return obs


@pytest.mark.parametrize("dtype,H,n,tol", [("f32", 64, 100, TOL_F32), ("f32", 256, 37, TOL_F32),
                                           ("bf16", 64, 50, TOL_BF16), ("bf16", 256, 300, TOL_BF16),
                                           ("f32", 512, 20, TOL_F32), ("bf16", 32, 17, TOL_BF16)])
def test_ensemble_act_matches_oracle(dtype, H, n, tol):
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble
    dev = cuda()
    print(f"[act] {dtype} H={H} n={n}", flush=True)
    obs = _obs_sample(n, 40 + H)
    acfg, actors, packed = actors_case(3, 211, H, 30)
    ens = Ensemble(packed, 3, 211, H, 30, dtype=dtype, max_batch=max(n, 64), device=dev)
    act, mean = ens.act(torch.from_numpy(obs).to(dev), t=3, sigma=0.1, noise_key=7, env_offset=10,
                        return_mean=True)
    w = device_weights(actors, dtype)
    ref_mean = ensemble_mean(w, obs)
    err = np.abs(_np(mean).astype(np.float64) - ref_mean)
    assert err.max() <= tol, f"mean off by {err.max():.3e}"
    from oracle.policy import ensemble_act
    ref_act = ensemble_act(w, obs, 3, 10, 0.1, 7)
    aerr = np.abs(_np(act).astype(np.float64) - ref_act.astype(np.float64))
    assert aerr.max() <= tol, f"action off by {aerr.max():.3e}"
    print(f"  mean err {err.max():.3e}  action err {aerr.max():.3e}", flush=True)


def test_ensemble_mix_weights_and_single_actor():
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble
    dev = cuda()
    obs = _obs_sample(40, 77)
    acfg, actors, packed = actors_case(3, 211, 64, 30)
    mix = np.array([0.2, 0.0, 0.8], np.float32)
    ens = Ensemble(packed, 3, 211, 64, 30, dtype="f32", max_batch=64, mix=mix, device=dev)
    _, mean = ens.act(torch.from_numpy(obs).to(dev), t=0, sigma=0.0, return_mean=True)
    ref = ensemble_mean(actors, obs, mix)
    assert np.abs(_np(mean) - ref).max() <= TOL_F32
    one = Ensemble(packed[: packed.size // 3], 1, 211, 64, 30, dtype="f32", max_batch=64, device=dev)
    _, m1 = one.act(torch.from_numpy(obs).to(dev), t=0, sigma=0.0, return_mean=True)
    assert np.abs(_np(m1) - ensemble_mean(actors[:1], obs)).max() <= TOL_F32


CLOSED = [
    # name, N, H, dtype, path, T, fused tuning (schedule, tile_envs), stocks
    ("plain f32 tiny", 16, 64, "f32", "plain", 30, (0, 0), 30),
    ("plain f32 ragged H=256", 37, 256, "f32", "plain", 12, (0, 0), 30),
    ("plain bf16", 24, 256, "bf16", "plain", 10, (0, 0), 30),
    ("fused bf16 tiny", 16, 64, "bf16", "fused", 30, (0, 0), 30),
    ("fused bf16 ragged H=256", 45, 256, "bf16", "fused", 12, (0, 0), 30),
    # The resident schedule with full and ragged tiles of 8, 5 and 3 environments, and the
    # streamed schedule, over more than one 64-day launch; 31 stocks (the resident limit) and 7.
    ("resident tiles of 8", 45, 256, "bf16", "fused", 70, (0, 8), 30),
    ("resident tiles of 5", 23, 256, "bf16", "fused", 20, (0, 5), 30),
    ("resident tiles of 3 D=31", 10, 256, "bf16", "fused", 20, (0, 3), 31),
    ("resident D=7", 19, 256, "bf16", "fused", 20, (0, 8), 7),
    # Launches of one and two days (the inputs of the first two days come with the set-up, later
    # ones are fetched two days ahead) after a full 64-day launch.
    ("resident 1-day launch", 13, 256, "bf16", "fused", 65, (0, 8), 30),
    ("resident 2-day launch", 11, 256, "bf16", "fused", 66, (0, 8), 30),
    ("streamed tiles of 16", 45, 256, "bf16", "fused", 70, (1, 16), 30),
]


@pytest.mark.parametrize("name,N,H,dtype,path,T,tuning,D", CLOSED, ids=[c[0] for c in CLOSED])
def test_closed_loop_rollout(name, N, H, dtype, path, T, tuning, D):
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    dev = cuda()
    print(f"[closed] {name}", flush=True)
    S = 7 * D + 1
    cfg, m = env_case(N, D, 5, T, 1001)
    acfg, actors, packed = actors_case(3, S, H, D)
    ens = Ensemble(packed, 3, S, H, D, dtype=dtype, max_batch=N, device=dev)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.set_fused_tuning(schedule=tuning[0], tile_envs=tuning[1])
    obs0 = _np(env.reset())
    traj = env.rollout(T, ens=ens, sigma=0.1, noise_key=7, path=path)
    traj = {k: _np(v) for k, v in traj.items()}
    check_replay(cfg, m, traj, obs0)
    tol = TOL_F32 if dtype == "f32" else TOL_BF16
    worst = check_actions(actors, dtype, traj, obs0, 0.1, 7, tol)
    assert np.abs(traj["qty"]).sum() > 0
    print(f"  worst action error {worst:.3e}", flush=True)


@pytest.mark.parametrize("H", [64, 256])
def test_fused_rollout_resumes_mid_trajectory(H):
    """Two fused launches (9 + 11 steps) give the same trajectory as one of 20 steps (generic
    schedule at H = 64, resident at 256)."""
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    dev = cuda()
    cfg, m = env_case(20, 30, 5, 20, 1001)
    acfg, actors, packed = actors_case(3, 211, H, 30)
    ens = Ensemble(packed, 3, 211, H, 30, dtype="bf16", max_batch=20, device=dev)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.reset(return_obs=False)
    full = env.rollout(20, ens=ens, sigma=0.1, noise_key=7, path="fused")
    env.reset(return_obs=False)
    a = env.rollout(9, ens=ens, sigma=0.1, noise_key=7, path="fused")
    b = env.rollout(11, ens=ens, sigma=0.1, noise_key=7, path="fused")
    for k in full:
        assert torch.equal(full[k], torch.cat([a[k], b[k]])), k
