"""Oracle trajectories: the closed loop replays exactly as a driven rollout."""
import numpy as np

from oracle.rollout import rollout_closed_loop, rollout_driven
from workload import TINY, make_actor_weights, make_market


def test_closed_loop_replays_as_driven():
    w = TINY
    cfg = w.env.replace(n_envs=8, n_days=12)
    m = make_market(w.market_seed, cfg.n_stocks, cfg.n_days)
    actors = make_actor_weights(w.actors.replace(bias_std=0.1))
    cl = rollout_closed_loop(cfg, m.close, m.ind, actors, cfg.n_days, w.sigma, w.noise_key)
    dr = rollout_driven(cfg, m.close, m.ind, cl["act"])
    for key in ("obs", "exec", "reward", "cash", "hold", "asset", "cumrew"):
        assert np.array_equal(cl[key], dr[key]), key
    assert cl["day"] == cfg.n_days
    assert cl["obs"].shape == (cfg.n_days + 1, 8, cfg.state_dim)
    # Noise makes trajectories differ across envs even on a shared market.
    assert len({cl["hold"][n].tobytes() for n in range(8)}) > 1
    # The policy actually trades.
    assert np.abs(cl["exec"]).sum() > 0
