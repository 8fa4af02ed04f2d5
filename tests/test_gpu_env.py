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


KERNELS = {0: "by-shape", 1: "tile", 2: "lane", 3: "row"}
DRIVEN = [c + (k,) for c in CASES for k in KERNELS if not (k >= 2 and c[2] > 32)]


@pytest.mark.parametrize("name,N,D,I,T,seed,extra,kernel", DRIVEN, ids=[f"{c[0]}-{KERNELS[c[-1]]}" for c in DRIVEN])
def test_driven_rollout_matches_oracle(name, N, D, I, T, seed, extra, kernel):
    """kernel 0 picks by shape and size (the tile kernel below 24576 environments), 1 the tile
    kernel, 2 the lane kernel (one lane per environment), 3 the row kernel (a 16-lane row per
    environment) where the shape allows (D <= 32)."""
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    print(f"[driven] {name} kernel {kernel}", flush=True)
    cfg, m = env_case(N, D, I, T, seed, **extra)
    acts = make_actions(seed + 100, T, N, D)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.set_step_kernel(kernel)
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


LANE = [
    # N, D, I, envs per wavefront (0: by N), T, cash, hmax
    (197, 30, 5, 64, 9, 1e6, 100),   # a partial last wavefront and workgroup
    (197, 30, 5, 3, 9, 1e6, 100),
    (130, 32, 5, 1, 7, 1e6, 100),    # 32 stocks: every register slot in use
    (90, 16, 4, 7, 8, 1e6, 100),
    (90, 9, 3, 0, 8, 1e6, 100),
    (50, 8, 2, 5, 8, 1e6, 100),
    (61, 30, 5, 0, 12, 4e3, 50),     # cash binds: partial fills on most days
]


@pytest.mark.parametrize("N,D,I,M,T,cash,hmax", LANE)
def test_lane_kernel_widths_match_oracle(N, D, I, M, T, cash, hmax):
    """The lane kernel at each register width (8, 16, 32 stocks) and wavefront width, driven by
    the same actions as the oracle: holdings, quantities, states and float64 cash bit-exact."""
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    print(f"[lane] N={N} D={D} I={I} M={M} T={T} cash={cash}", flush=True)
    cfg, m = env_case(N, D, I, T, 40 + D, hmax=hmax, cash=cash)
    acts = make_actions(77 + D, T, N, D)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.set_step_kernel(2, M)
    obs0 = _to_np(env.reset())
    traj = env.rollout(T, actions=torch.from_numpy(acts).to(dev))
    st = env.read_state()
    traj = {k: _to_np(v) for k, v in traj.items()}
    ref = check_replay(cfg, m, traj, obs0)
    assert np.array_equal(_to_np(st["hold"]), ref["hold"])
    assert np.array_equal(_to_np(st["cash"]), ref["cash"])
    assert np.array_equal(_to_np(st["asset"]), ref["asset"])
    assert np.abs(traj["qty"]).sum() > 0


def test_driven_large_batch_by_shape_sampled():
    """30011 environments: the size-based choice takes the lane kernel (30 environments per
    wavefront, the last wavefront ragged); a sample including the wavefront edges is replayed."""
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    N, D, T = 30011, 30, 4
    cfg, m = env_case(N, D, 5, T, 9)
    acts = make_actions(109, T, N, D)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    obs0 = _to_np(env.reset())
    traj = env.rollout(T, actions=torch.from_numpy(acts).to(dev))
    traj = {k: _to_np(v) for k, v in traj.items()}
    ids = [0, 1, 29, 30, 31, 15000, 29999, 30000, 30001, 30009, 30010]
    check_replay(cfg, m, traj, obs0, env_ids=ids)


def test_lane_kernel_plain_steps_match_tile_kernel():
    """The plain path's ensemble steps (mean of the actors, noise, clip, trade) through the lane
    kernel and through the tile kernel: the same arithmetic, so every output is bit-identical.
    The lane kernel stages the actors' means through LDS for small wavefront tiles (1 and 5
    environments) and reads them into registers for a full 64-environment tile; the row kernel
    takes them per lane (one or two environments per wavefront).  N = 77: the last wavefront of the
    two-environment row kernel holds one environment."""
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    from _helpers import actors_case
    dev = cuda()
    N, D, T = 77, 30, 12
    cfg, m = env_case(N, D, 5, T, 1001)
    _, _, packed = actors_case(3, 211, 64, D)
    ens = Ensemble(packed, 3, 211, 64, D, dtype="f32", max_batch=N, device=dev)
    out = []
    for kernel, M in ((1, 0), (2, 0), (2, 5), (2, 64), (3, 0), (3, 1)):
        env = VecEnv(cfg, m.close, m.ind, device=dev)
        env.set_step_kernel(kernel, M)
        env.reset(return_obs=False)
        out.append(env.rollout(T, ens=ens, sigma=0.1, noise_key=7, path="plain"))
    for other in out[1:]:
        for k in out[0]:
            assert torch.equal(out[0][k], other[k]), k


ROW = [
    # N, D, I, T, cash, hmax
    (31, 30, 5, 9, 1e6, 100),    # the last wavefront holds one environment
    (20, 32, 5, 7, 1e6, 100),    # 32 stocks: both stock slots of every lane in use
    (18, 17, 4, 8, 1e6, 100),
    (9, 3, 2, 8, 1e6, 100),
    (33, 30, 5, 12, 4e3, 50),    # cash binds: partial fills on most days
    (258, 32, 3, 16, 3e4, 100),  # cash binds after a few days: runs of whole fills then partials
]


@pytest.mark.parametrize("envs_per_wave", [1, 2])
@pytest.mark.parametrize("N,D,I,T,cash,hmax", ROW)
def test_row_kernel_matches_oracle(N, D, I, T, cash, hmax, envs_per_wave):
    """The row kernel (one or two environments per wavefront) driven by the same actions as the
    oracle: holdings, quantities, states and float64 cash bit-exact."""
    import torch
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    print(f"[row] N={N} D={D} I={I} T={T} cash={cash} envs_per_wave={envs_per_wave}", flush=True)
    cfg, m = env_case(N, D, I, T, 60 + D, hmax=hmax, cash=cash)
    acts = make_actions(97 + D, T, N, D)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    env.set_step_kernel(3, envs_per_wave)
    obs0 = _to_np(env.reset())
    traj = env.rollout(T, actions=torch.from_numpy(acts).to(dev))
    st = env.read_state()
    traj = {k: _to_np(v) for k, v in traj.items()}
    ref = check_replay(cfg, m, traj, obs0)
    assert np.array_equal(_to_np(st["hold"]), ref["hold"])
    assert np.array_equal(_to_np(st["cash"]), ref["cash"])
    assert np.array_equal(_to_np(st["asset"]), ref["asset"])
    assert np.abs(traj["qty"]).sum() > 0


def test_step_kernel_choice_validation():
    from paper_2501_10709_amd.vecenv import VecEnv
    dev = cuda()
    cfg, m = env_case(8, 40, 5, 4, 3)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    with pytest.raises(RuntimeError):
        env.set_step_kernel(2)  # 40 stocks: beyond the lane kernel
    with pytest.raises(RuntimeError):
        env.set_step_kernel(3)  # also beyond the row kernel
    with pytest.raises(RuntimeError):
        env.set_step_kernel(4)
    env.set_step_kernel(0)
    cfg, m = env_case(8, 30, 5, 4, 3)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    with pytest.raises(RuntimeError):
        env.set_step_kernel(3, 3)  # the row kernel holds one or two environments per wavefront
    env.set_step_kernel(3, 1)


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
