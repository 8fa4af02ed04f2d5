"""Pins of the crypto oracle (oracle/crypto.py) to values fixed by the paper's definitions and by
mathematics: a hand-worked three-tick trajectory, telescoping identities of the reward, brute force
over every action sequence of a short horizon, closed forms of the ReLU network, softmax and vote
rules, and the exploration generator's frequencies."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import crypto as oc
from workload.crypto import N_FEAT, TickMarket, WARMUP, crypto_actors, make_ticks, place, poisson_requests
from workload import make_actor_weights

GOLD = os.path.join(os.path.dirname(__file__), "golden", "crypto_hand_worked.json")


def _market(mid):
    mid = np.asarray(mid, np.float64)
    return TickMarket(mid=mid, feat=np.zeros((mid.size, N_FEAT), np.float32))


def test_hand_worked_three_ticks():
    g = json.load(open(GOLD))
    st = oc.CryptoState(1, g["cash0"])
    mid = g["mid"]
    for t, (a, want) in enumerate(zip(g["actions"], g["steps"])):
        r = oc.step(st, np.array([a]), np.array([mid[t]]), np.array([mid[t + 1]]), g["fee"])
        assert st.cash[0] == float.fromhex(want["cash"])
        assert st.pos[0] == want["pos"]
        assert st.value[0] == float.fromhex(want["value"])
        assert r[0] == float.fromhex(want["reward"])
    f = g["final"]
    for k in ("sum_r", "sum_r2", "peak", "mdd"):
        assert getattr(st, k)[0] == float.fromhex(f[k]), k
    assert st.trades[0] == f["trades"]


def test_rewards_telescope_to_position_pnl_minus_fees():
    """sum_t r_t = sum_t h'_t (p_{t+1} - p_t) - sum_t |Delta_t| p_t fee (exact in rationals)."""
    rng = np.random.default_rng(3)
    mid = 50_000 * np.exp(np.cumsum(rng.standard_normal(201) * 1e-3))
    acts = rng.integers(0, 3, size=(200, 7))
    st = oc.CryptoState(7, 1e5)
    total = np.zeros(7)
    for t in range(200):
        total += oc.step(st, acts[t], np.full(7, mid[t]), np.full(7, mid[t + 1]), 2e-4)
    pos = acts - 1
    prev = np.vstack([np.zeros((1, 7), int), pos[:-1]])
    pnl = (pos * (mid[1:, None] - mid[:-1, None])).sum(0)
    fees = (np.abs(pos - prev) * mid[:-1, None] * 2e-4).sum(0)
    np.testing.assert_allclose(total, pnl - fees, rtol=0, atol=1e-7)
    np.testing.assert_allclose(st.value - 1e5, pnl - fees, rtol=0, atol=1e-7)
    assert (st.trades == (pos != prev).sum(0)).all()


def test_flat_policy_keeps_cash():
    m = _market(50_000 + 10 * np.arange(20))
    st = oc.CryptoState(3, 1e5)
    for t in range(19):
        r = oc.step(st, np.ones(3, int), np.full(3, m.mid[t]), np.full(3, m.mid[t + 1]), 2e-4)
        assert (r == 0).all()
    assert (st.cash == 1e5).all() and (st.trades == 0).all() and (st.mdd == 0).all()


def test_statistics_brute_force_over_all_action_sequences():
    """Every action sequence of 4 ticks: peak, max drawdown and sums against direct formulas on
    the value path."""
    mid = np.array([50_000.0, 50_400.0, 49_700.0, 50_100.0, 49_900.0])
    seqs = np.array(list(itertools.product(range(3), repeat=4)))   # [81][4]
    st = oc.CryptoState(len(seqs), 1e5)
    vals = [st.value.copy()]
    rs = []
    for t in range(4):
        rs.append(oc.step(st, seqs[:, t], np.full(len(seqs), mid[t]), np.full(len(seqs), mid[t + 1]), 2e-4))
        vals.append(st.value.copy())
    V = np.stack(vals)   # [5][81]
    for i in range(len(seqs)):
        v = V[:, i]
        mdd = max(v[a] - v[b] for a in range(5) for b in range(a, 5))
        assert st.mdd[i] == pytest.approx(mdd, abs=1e-9)
        assert st.peak[i] == v.max()
        assert st.sum_r[i] == pytest.approx(v[-1] - v[0], abs=1e-9)
        assert st.sum_r2[i] == pytest.approx(sum(float(r[i]) ** 2 for r in rs), rel=1e-12)


def test_state_row_layout():
    f = np.arange(2 * N_FEAT, dtype=np.float32).reshape(2, N_FEAT)
    x = oc.state_rows(np.array([131072.0, 1e5]), np.array([-1, 1]), np.array([65536.0, 50_000.0]), f)
    assert x.dtype == np.float32
    assert x[0, 0] == 1.0 and x[0, 1] == 1.0 and x[0, 2] == -1.0
    assert x[1, 0] == np.float32(1e5 / 131072.0) and x[1, 2] == 1.0
    assert (x[:, 3:] == f[:, 3:]).all()


def _abs_net():
    """W1 routes x[3] to h1 = (relu(x3), relu(-x3)); W2 copies; W3 gives Q = (|x3|, 0, -|x3|) + b3."""
    p = {"W1": np.zeros((16, 128), np.float32), "b1": np.zeros(128, np.float32),
         "W2": np.zeros((128, 128), np.float32), "b2": np.zeros(128, np.float32),
         "W3": np.zeros((128, 3), np.float32), "b3": np.array([0.0, 0.0, 0.5], np.float32)}
    p["W1"][3, 0], p["W1"][3, 1] = 1.0, -1.0
    p["W2"][0, 5], p["W2"][1, 6] = 1.0, 1.0
    p["W3"][5, 0], p["W3"][6, 0] = 1.0, 1.0
    p["W3"][5, 2], p["W3"][6, 2] = -1.0, -1.0
    return p


def test_relu_network_closed_form():
    x = np.zeros((5, 16), np.float32)
    x[:, 3] = [-2.0, -0.5, 0.0, 0.25, 3.0]
    q = oc.q_values(_abs_net(), x)
    a = np.abs(x[:, 3].astype(np.float64))
    np.testing.assert_array_equal(q, np.stack([a, 0 * a, 0.5 - a], 1))


def test_softmax_average_rules():
    rng = np.random.default_rng(1)
    actors = make_actor_weights(crypto_actors(n_actors=3))
    x = rng.standard_normal((50, 16)).astype(np.float32)
    p = oc.ensemble_probs(actors, x)
    np.testing.assert_allclose(p.sum(1), 1.0, atol=1e-15)
    # K=1 reduces to that agent's softmax; one-hot weights select an agent.
    q0 = oc.q_values(actors[0], x)
    e = np.exp(q0 - q0.max(1, keepdims=True))
    np.testing.assert_allclose(oc.ensemble_probs(actors[:1], x), e / e.sum(1, keepdims=True), rtol=1e-15)
    np.testing.assert_allclose(oc.ensemble_probs(actors, x, mix=[0, 1, 0]), oc.ensemble_probs(actors[1:2], x),
                               rtol=1e-15)
    # Softmax is invariant to a shift of all Q-values (the output bias adds a constant).
    shifted = [dict(a, b3=a["b3"].astype(np.float64) + 3.0) for a in actors]
    np.testing.assert_allclose(oc.ensemble_probs(shifted, x), p, rtol=1e-12)


def test_argmax_and_vote_ties_go_to_lowest_index():
    assert list(oc.first_argmax(np.array([[1, 1, 0], [0, 2, 2], [3, 3, 3]]))) == [0, 1, 0]
    # Three agents with Q = (|x|,0,0.5-|x|), (0,1,0), (0,0,1): at x=0 the votes are 2, 1, 2 -> 2;
    # at |x| large: 0, 1, 2 -> a three-way tie -> 0.
    a0 = _abs_net()
    a1 = dict(_abs_net(), W3=np.zeros((128, 3), np.float32), b3=np.array([0, 1, 0], np.float32))
    a2 = dict(_abs_net(), W3=np.zeros((128, 3), np.float32), b3=np.array([0, 0, 1], np.float32))
    x = np.zeros((2, 16), np.float32)
    x[1, 3] = 5.0
    assert list(oc.vote_actions([a0, a1, a2], x)) == [2, 0]


def test_exploration_frequencies_and_independence():
    explore, rand = oc.exploration(0xABC, np.arange(200_000), 17, 0.05)
    assert abs(explore.mean() - 0.05) < 4 * math.sqrt(0.05 * 0.95 / 200_000)
    counts = np.bincount(rand, minlength=3) / rand.size
    assert np.abs(counts - 1 / 3).max() < 0.005
    e2, _ = oc.exploration(0xABC, np.arange(200_000), 18, 0.05)
    assert abs((explore & e2).mean() - 0.0025) < 0.0006     # steps draw independently
    assert not oc.exploration(0xABC, np.arange(1000), 0, 0.0)[0].any()
    assert oc.exploration(0xABC, np.arange(1000), 0, 1.0)[0].all()


def test_closed_loop_flat_when_middle_action_dominates():
    """Agents whose Q strongly favour action 1 keep every environment flat without exploration."""
    p = {"W1": np.zeros((16, 128), np.float32), "b1": np.zeros(128, np.float32),
         "W2": np.zeros((128, 128), np.float32), "b2": np.zeros(128, np.float32),
         "W3": np.zeros((128, 3), np.float32), "b3": np.array([0, 4, 0], np.float32)}
    m = make_ticks(seed=2, n_ticks=400)
    st, probs, chosen, greedy, explored, rew = oc.rollout(m, [p, p], 3, 50, WARMUP, 5, key=1, eps=0.0)
    assert (chosen == 1).all() and (rew == 0).all() and (st["cash"] == 1e5).all()
    np.testing.assert_allclose(probs[..., 1], math.exp(4) / (math.exp(4) + 2), rtol=1e-15)


def test_driven_rollout_matches_closed_loop_on_its_own_actions():
    m = make_ticks(seed=5, n_ticks=2000)
    actors = make_actor_weights(crypto_actors())
    a = oc.rollout(m, actors, 6, 40, 100, 13, key=9, eps=0.1)
    b = oc.rollout(m, actors, 6, 40, 100, 13, key=9, eps=0.1, actions=a[2])
    for k in a[0]:
        np.testing.assert_array_equal(a[0][k], b[0][k])
    np.testing.assert_array_equal(a[1], b[1])
    assert a[4].any() and not a[4].all()


def test_tick_generator_features():
    m = make_ticks(seed=7, n_ticks=5000)
    r = np.diff(np.log(m.mid))
    t = 1000
    np.testing.assert_allclose(m.feat[t, 3:13], (r[t - 10:t][::-1] * 1e4), rtol=1e-5)
    np.testing.assert_allclose(m.feat[t, 13], np.std(r[t - 10:t]) * 1e4, rtol=1e-4)
    np.testing.assert_allclose(m.feat[t, 14], np.std(r[t - 60:t]) * 1e4, rtol=1e-4)
    assert (m.feat[:, :3] == 0).all() and np.abs(m.feat[:, 15]).max() <= 1.0
    # Student-t(3)/sqrt(3) * 1e-4: median |r| of t3 is 0.7649 (t3 quantile 0.75), so 0.4416e-4.
    assert abs(np.median(np.abs(r)) / 1e-4 - 0.7649 / math.sqrt(3)) < 0.03


def test_request_placement_stays_inside_the_table():
    reqs = poisson_requests(3, 300, 200.0, 1_000_000)
    for q in reqs:
        last = q.start_tick + q.stride * (q.n_envs - 1) + q.horizon
        assert q.start_tick >= WARMUP and last <= 1_000_000 - 1
        assert 1 <= q.n_envs <= 4096 and 1000 <= q.horizon <= 100_000
    gaps = np.diff([0.0] + [q.arrival_s for q in reqs])
    assert abs(gaps.mean() - 1 / 200) < 0.2 / 200
    rng = np.random.default_rng(0)
    assert place(rng, 1, 10, 200) [1] == 0
