"""GPU environment kernels against the CPU oracle, driven by identical actions.

Holdings, executed quantities and the float32 states must be bit-exact; cash, total asset and
rewards are float64 and must agree within 1e-12 relative (the kernels keep the oracle's order of
operations, so they are in fact bit-exact and the test records that too).
"""
import numpy as np
import pytest

from _helpers import TOL_F64_REL, assert_f64_close, check_replay, cuda, env_case
from oracle.env import OracleEnv
from oracle.rollout import rollout_driven
from workload import make_actions

pytestmark = pytest.mark.gpu

CASES = [
    # name, N, D, I, T, seed, extra
    ("tiny N=16 D=30 T=30", 16, 30, 5, 30, 1, {}),
    ("ragged N=37", 37, 30, 5, 20, 2, {}),
    ("D=7 I=3", 70, 7, 3, 15, 3, {}),
    ("D=100 I=2", 9, 100, 2, 10, 4, {}),
    ("D=50", 33, 50, 5, 10, 5, {}),
    ("D=2 cash binds", 20, 2, 1, 12, 6, dict(hmax=3, cash=300.0)),
    ("N=5000 tiles of 16", 5000, 30, 5, 6, 7, {}),
    ("D=1 I=0", 11, 1, 0, 9, 8, dict(cost=0.0)),
]


def _to_np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,N,D,I,T,seed,extra", CASES, ids=[c[0] for c in CASES])
def test_driven_rollout_matches_oracle(name, N, D, I, T, seed, extra):
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    print(f"[driven] {name}", flush=True)
    cfg, m = env_case(N, D, I, T, seed, **extra)
    acts = make_actions(seed + 100, T, N, D)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    obs0 = _to_np(env.reset())
    traj = env.rollout(T, actions=torch.from_numpy(acts).to(dev))
    st = env.read_state()
    torch.cuda.synchronize()
    traj = {k: _to_np(v) for k, v in traj.items()}
    assert np.array_equal(traj["act"], acts)
    ref = check_replay(cfg, m, traj, obs0)
    assert np.array_equal(_to_np(st["hold"]), ref["hold"])
    assert_f64_close(_to_np(st["cash"]), ref["cash"], ref["asset"], "cash")
    assert_f64_close(_to_np(st["asset"]), ref["asset"], ref["asset"], "asset")
    assert_f64_close(_to_np(st["cumrew"]), ref["cumrew"], ref["asset"] * cfg.reward_scale * T, "cumrew")
    assert st["day"] == T
    # Same operation order as the oracle: bit-exact float64 too.
    assert np.array_equal(_to_np(st["cash"]), ref["cash"])
    assert np.array_equal(_to_np(st["asset"]), ref["asset"])


def test_step_api_matches_oracle_and_reports_done():
    import torch
    from paper_2501_10709_amd import FmError
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    cfg, m = env_case(21, 30, 5, 8, 11)
    acts = make_actions(12, 8, 21, 30)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    ora = OracleEnv(cfg, m.close, m.ind)
    assert np.array_equal(_to_np(env.reset()), ora.reset())
    for t in range(8):
        obs, rew, qty, done = env.step(torch.from_numpy(acts[t]).to(dev))
        o_obs, o_rew, o_qty, o_done = ora.step(acts[t])
        assert np.array_equal(_to_np(obs), o_obs)
        assert np.array_equal(_to_np(qty), o_qty)
        assert np.array_equal(_to_np(rew), o_rew)
        assert done == o_done == (t == 7)
    with pytest.raises(FmError) as e:
        env.step(torch.from_numpy(acts[0]).to(dev))
    assert e.value.status == 2
    # Reset brings it back.
    assert np.array_equal(_to_np(env.reset()), ora.reset())
    assert env.day == 0


def test_special_actions_nan_inf_and_out_of_range():
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    cfg, m = env_case(6, 30, 5, 3, 13)
    a = make_actions(14, 3, 6, 30)
    a[0, 0, :5] = [np.nan, np.inf, -np.inf, 7.5, -3.0]
    a[1, 1, :4] = [np.nan, 2.0, -2.0, 1e30]
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    obs0 = _to_np(env.reset())
    traj = {k: _to_np(v) for k, v in env.rollout(3, actions=torch.from_numpy(a).to(dev)).items()}
    check_replay(cfg, m, traj, obs0)


def test_state_write_resumes_bit_identically():
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    cfg, m = env_case(40, 30, 5, 20, 15)
    acts = torch.from_numpy(make_actions(16, 20, 40, 30)).to(dev)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.reset(return_obs=False)
    env.rollout(9, actions=acts[:9])
    snap = env.read_state()
    tail_a = env.rollout(11, actions=acts[9:])
    env2 = VecEnv(cfg, m.close, m.ind, device=dev)
    env2.write_state(snap)
    assert env2.day == 9
    tail_b = env2.rollout(11, actions=acts[9:])
    for k in tail_a:
        assert torch.equal(tail_a[k], tail_b[k]), k
    # Oracle continuation from the same snapshot.
    ora = OracleEnv(cfg, m.close, m.ind)
    ora.set_state({k: (_to_np(v) if hasattr(v, "cpu") else v) for k, v in snap.items()})
    for i, t in enumerate(range(9, 20)):
        o, r, x, _ = ora.step(_to_np(acts[t]))
        assert np.array_equal(_to_np(tail_a["obs"][i]), o)
        assert np.array_equal(_to_np(tail_a["qty"][i]), x)


def test_rollout_past_horizon_is_a_state_error():
    import torch
    from paper_2501_10709_amd import FmError
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    cfg, m = env_case(4, 30, 5, 5, 17)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.reset(return_obs=False)
    acts = torch.zeros((6, 4, 30), dtype=torch.float32, device=dev)
    with pytest.raises(FmError) as e:
        env.rollout(6, actions=acts)
    assert e.value.status == 2
    env.rollout(5, actions=acts[:5])
    with pytest.raises(FmError):
        env.rollout(1, actions=acts[:1])
    env.rollout(0, actions=acts[:0])  # zero steps is a no-op
