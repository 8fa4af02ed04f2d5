"""Checks on the seeded synthetic inputs (market, indicators, actors, actions)."""
import numpy as np

from workload import (PAPER_SCALE, TINY, ActorConfig, make_actions, make_actor_weights, make_market,
                      pack_actor_weights, state_width, unpack_actor_weights)
from workload.market import _rolling_mean, _rsi_wilder, gbm_closes


def test_state_width():
    assert state_width(30, 5) == 211
    assert [state_width(d, 5) for d in (5, 10, 50, 100)] == [36, 71, 351, 701]
    assert TINY.env.state_dim == 211 == PAPER_SCALE.actors.in_dim


def test_gbm_mean_matches_closed_form():
    rng = np.random.default_rng(0)
    s = gbm_closes(rng, 50, 20000, 3e-4, 0.02)
    ratio = s[-1] / s[0]
    expect = np.exp(3e-4 * 50)
    se = ratio.std() / np.sqrt(ratio.size)
    assert abs(ratio.mean() - expect) < 5 * se


def test_indicator_identities():
    const = np.full((40, 3), 7.0)
    assert np.allclose(_rolling_mean(const, 5), 7.0)
    rising = np.cumsum(np.ones((40, 2)), axis=0)
    assert np.allclose(_rsi_wilder(rising)[1:], 100.0)
    m = make_market(3, 30, 252)
    rsi = (m.ind[:, 2, :] + 0.5) * 100
    assert np.all((rsi >= 0) & (rsi <= 100))


def test_market_shapes_and_determinism():
    a = make_market(1001, 30, 30)
    b = make_market(1001, 30, 30)
    assert a.close.shape == (31, 30) and a.ind.shape == (31, 5, 30)
    assert a.close.dtype == np.float32 and a.ind.dtype == np.float32
    assert a.close.tobytes() == b.close.tobytes() and a.ind.tobytes() == b.ind.tobytes()
    assert np.all(a.close > 0) and np.all(np.isfinite(a.ind))
    assert np.all(a.high >= a.low)
    assert make_market(1002, 30, 30).close.tobytes() != a.close.tobytes()


def test_actor_pack_roundtrip_and_xavier_limits():
    cfg = ActorConfig(n_actors=3, in_dim=211, hidden=64, out_dim=30)
    actors = make_actor_weights(cfg)
    flat = pack_actor_weights(actors)
    assert flat.size == 3 * (211 * 64 + 64 + 64 * 64 + 64 + 64 * 30 + 30)
    back = unpack_actor_weights(flat, cfg)
    for p, q in zip(actors, back):
        for k in p:
            assert np.array_equal(p[k], q[k])
    lim = np.sqrt(6.0 / (211 + 64))
    assert np.abs(actors[0]["W1"]).max() <= lim and np.abs(actors[0]["W1"]).max() > 0.9 * lim
    assert not actors[0]["b1"].any()
    assert not np.array_equal(actors[0]["W1"], actors[1]["W1"])


def test_actions_cover_special_values():
    a = make_actions(9, 10, 64, 30)
    assert a.dtype == np.float32 and a.shape == (10, 64, 30)
    assert np.all(np.abs(a) <= 1)
    assert (a == 0).any() and (a == 1).any() and (a == -1).any()
    assert ((np.abs(a) < 0.01) & (a != 0)).any()


def test_uneven_groups_follow_their_recipe():
    import math
    from workload.uneven import uneven_groups
    gs = uneven_groups(seed=4, n_groups=64)
    assert len(gs) == 64
    assert {g.env.n_stocks for g in gs} <= {5, 10, 30, 50, 100}
    assert all(32 <= g.env.n_envs <= 4096 and 20 <= g.env.n_days <= 1000 for g in gs)
    assert all(0.01 <= g.vol <= 0.04 for g in gs)
    assert all(g.actors.in_dim == 7 * g.env.n_stocks + 1 and g.actors.out_dim == g.env.n_stocks for g in gs)
    # log-uniform env counts: the median of log N sits near the middle of [log 32, log 4096]
    med = float(np.median([math.log(g.env.n_envs) for g in gs]))
    assert abs(med - 0.5 * (math.log(32) + math.log(4096))) < 0.9
    assert uneven_groups(seed=4, n_groups=64) == gs  # seeded
