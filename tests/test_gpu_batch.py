"""Uneven batch (groups with their own stock count, environment count, horizon and ensemble,
stepped together by the batched persistent kernel) against the oracle, graph replays against
the eager run, and the autotuner leaving the state untouched."""
import numpy as np
import pytest

from _helpers import TOL_BF16, actors_case, check_actions, check_replay, cuda, env_case

pytestmark = pytest.mark.gpu

# (D, N, T, seed): stock counts 5..50, ragged env counts, horizons over one and two 64-day chunks.
GROUPS = [(5, 20, 70, 11), (10, 37, 25, 12), (30, 64, 40, 13), (50, 16, 66, 14), (7, 50, 20, 15), (30, 33, 64, 16)]
H = 64


def _np(t):
    return t.detach().cpu().numpy()


def _build(dev):
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    made = []
    for D, N, T, seed in GROUPS:
        cfg, m = env_case(N, D, 5, T, seed)
        S = 7 * D + 1
        acfg, actors, packed = actors_case(3, S, H, D, seed_base=100 * seed)
        ens = Ensemble(packed, 3, S, H, D, dtype="bf16", max_batch=N, device=dev)
        env = VecEnv(cfg, m.close, m.ind, device=dev)
        made.append((cfg, m, actors, ens, env))
    return made


def _spec(made, store=("obs", "act", "rew", "qty")):
    return [dict(env=env, ens=ens, n_steps=cfg.n_days, sigma=0.1, noise_key=7, env_offset=1000 * i, store=store)
            for i, (cfg, m, actors, ens, env) in enumerate(made)]


def test_batch_matches_oracle():
    from paper_2501_10709_amd.vecenv import Batch
    dev = cuda()
    made = _build(dev)
    obs0 = [_np(env.reset()) for *_, env in made]
    batch = Batch(_spec(made))
    out = batch.run()
    for i, (cfg, m, actors, ens, env) in enumerate(made):
        print(f"[batch] group {i} D={cfg.n_stocks} N={cfg.n_envs} T={cfg.n_days}", flush=True)
        traj = {k: _np(v) for k, v in out[i].items()}
        check_replay(cfg, m, traj, obs0[i])
        worst = check_actions(actors, "bf16", traj, obs0[i], 0.1, 7, TOL_BF16, env_offset=1000 * i)
        assert env.day == cfg.n_days
        assert np.abs(traj["qty"]).sum() > 0
        print(f"  worst action error {worst:.3e}", flush=True)
    batch.close()


def test_graph_replays_and_tuning_match_eager():
    import torch
    from paper_2501_10709_amd.vecenv import Batch
    dev = cuda()
    made = _build(dev)
    for *_, env in made:
        env.reset(return_obs=False)
    batch = Batch(_spec(made, store=("rew", "qty")))
    eager = [{k: v.clone() for k, v in o.items()} for o in batch.run(use_graph=False)]
    for rep in range(3):
        for *_, env in made:
            env.reset(return_obs=False)
        junk = torch.randn(1 << 20, device=dev).sum()  # eager work between replays
        torch.cuda.synchronize()
        out = batch.run(use_graph=True)
        torch.cuda.synchronize()
        for g, (o, e) in enumerate(zip(out, eager)):
            for k in e:
                assert torch.equal(o[k], e[k]), (rep, g, k)
        del junk
    # The autotuner restores the states it runs on, and its choice gives the same results.
    for *_, env in made:
        env.reset(return_obs=False)
    before = [env.read_state() for *_, env in made]
    rows, blocks = batch.tune()
    assert rows in (16, 32) and blocks > 0
    after = [env.read_state() for *_, env in made]
    for a, b in zip(before, after):
        for k in a:
            if isinstance(a[k], torch.Tensor):
                assert torch.equal(a[k], b[k]), k
    out = batch.run(use_graph=True)
    for g, (o, e) in enumerate(zip(out, eager)):
        for k in e:
            assert torch.equal(o[k], e[k]), ("tuned", g, k)
    batch.close()


def test_batch_requires_recorded_days():
    from paper_2501_10709_amd import binding as B
    from paper_2501_10709_amd.vecenv import Batch
    dev = cuda()
    made = _build(dev)[:2]
    for *_, env in made:
        env.reset(return_obs=False)
    batch = Batch(_spec(made, store=("rew",)))
    batch.run()
    with pytest.raises(B.FmError):
        batch.run()  # the environments are no longer at their starting days
    batch.close()


# Hidden width 256 (every MLP wavefront walks four output tiles per layer), wide groups (D = 100:
# state width 701) and horizons over three and more 64-day chunks, as the benchmark's batch has.
GROUPS_256 = [(100, 20, 130, 21), (30, 40, 140, 22), (50, 17, 70, 23), (5, 70, 20, 24), (30, 33, 200, 25)]


def _build_256(dev, groups):
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    made = []
    for D, N, T, seed in groups:
        cfg, m = env_case(N, D, 5, T, seed)
        S = 7 * D + 1
        acfg, actors, packed = actors_case(3, S, 256, D, seed_base=100 * seed)
        ens = Ensemble(packed, 3, S, 256, D, dtype="bf16", max_batch=N, device=dev)
        env = VecEnv(cfg, m.close, m.ind, device=dev)
        made.append((cfg, m, actors, ens, env))
    return made


@pytest.mark.parametrize("tiling", ["tuned", (16, 128), (16, 512), (32, 256)])
def test_batch_hidden_256_matches_oracle(tiling):
    """The benchmark's shapes under the autotuner's choice and under forced tilings, each run
    eagerly and then replayed from its graph: the eager run against the oracle (states and
    quantities exact, rewards 1e-12, actions 2e-2), the replay bit for bit against the eager run.
    Under 32-row tiling the D = 100 group, whose 32-row tile does not fit the LDS, keeps 16 rows
    in a launch of its own beside the 32-row groups."""
    import torch
    from paper_2501_10709_amd.vecenv import Batch
    dev = cuda()
    made = _build_256(dev, GROUPS_256)
    for *_, env in made:
        env.reset(return_obs=False)
    spec = [dict(env=env, ens=ens, n_steps=cfg.n_days, sigma=0.1, noise_key=9, env_offset=5000 * i,
                 store=("obs", "act", "rew", "qty")) for i, (cfg, m, actors, ens, env) in enumerate(made)]
    batch = Batch(spec)
    if tiling == "tuned":
        rows, blocks = batch.tune()
    else:
        rows, blocks = tiling
        batch.set_tiling(rows, blocks)
    print(f"[batch256] rows {rows} blocks {blocks} groups {len(made)}", flush=True)
    obs0 = [_np(env.reset()) for *_, env in made]
    out = batch.run(use_graph=False)
    torch.cuda.synchronize()
    eager = [{k: v.clone() for k, v in o.items()} for o in out]
    for i, (cfg, m, actors, ens, env) in enumerate(made):
        traj = {k: _np(v) for k, v in eager[i].items()}
        check_replay(cfg, m, traj, obs0[i])
        worst = check_actions(actors, "bf16", traj, obs0[i], 0.1, 9, TOL_BF16, env_offset=5000 * i)
        assert np.abs(traj["qty"]).sum() > 0
        print(f"  group {i} D={cfg.n_stocks} N={cfg.n_envs} T={cfg.n_days}: worst action error {worst:.3e}",
              flush=True)
    for *_, env in made:
        env.reset(return_obs=False)
    out = batch.run(use_graph=True)
    torch.cuda.synchronize()
    for g, (o, e) in enumerate(zip(out, eager)):
        for k in e:
            assert torch.equal(o[k], e[k]), (g, k)
    batch.close()
