"""Pins of the learner oracle (oracle/learner.py): its gradient against central finite differences of
the objective it differentiates, and closed forms of eqs. (4) and (5)."""
import numpy as np
import pytest

from oracle import learner as L
from workload import ActorConfig, make_actor_weights


def _case(K=2, S=5, H=4, A=3, T=3, N=4, seed=0):
    actors = make_actor_weights(ActorConfig(n_actors=K, in_dim=S, hidden=H, out_dim=A, seed_base=50 + seed,
                                            bias_std=0.2))
    rng = np.random.default_rng(seed)
    states = rng.standard_normal((T, N, S)).astype(np.float32)
    rewards = rng.standard_normal((T, N)) * 0.01
    return actors, states, rewards


@pytest.mark.parametrize("i,lam", [(0, 0.0), (1, 0.0), (0, 0.7), (1, 2.5)])
def test_gradient_matches_central_differences(i, lam):
    actors, states, rewards = _case()
    sigma, key, off = 0.1, 7, 3
    acts = L.sampled_actions(actors, states, sigma, key, off)
    R = L.returns(rewards)
    g = L.policy_gradient(actors, i, states, rewards, sigma, key, off, lam)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        base = np.asarray(actors[i][name], np.float64)
        fd = np.zeros_like(base)
        for idx in np.ndindex(base.shape):
            vals = []
            for sgn in (1, -1):
                pert = [dict((k, np.asarray(v, np.float64)) for k, v in a.items()) for a in actors]
                pert[i][name] = base.copy()
                pert[i][name][idx] += sgn * h
                vals.append(L.objective(pert, i, states, acts, R, sigma, lam))
            fd[idx] = (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(g[name], fd, rtol=2e-5, atol=1e-7 * max(1.0, np.abs(fd).max()), err_msg=name)


def test_zero_returns_and_no_diversity_give_zero():
    actors, states, _ = _case()
    g = L.policy_gradient(actors, 0, states, np.zeros((3, 4)), 0.1, 7, 0, 0.0)
    for v in g.values():
        assert np.abs(v).max() == 0.0


def test_identical_agents_have_no_diversity_gradient():
    actors, states, _ = _case(K=1)
    twins = [actors[0], dict(actors[0])]
    g = L.policy_gradient(twins, 0, states, np.zeros((3, 4)), 0.1, 7, 0, 5.0)
    for v in g.values():
        assert np.abs(v).max() == 0.0


def test_output_bias_gradient_closed_form():
    """For one agent (abar = mu), a - mu = sigma eps, so d/db3 = (1/N) sum R_n eps (1 - mu^2) / sigma."""
    actors, states, rewards = _case(K=1)
    sigma, key, off = 0.25, 11, 0
    g = L.policy_gradient(actors, 0, states, rewards, sigma, key, off, 0.0)
    T, N, S = states.shape
    acts = L.sampled_actions(actors, states, sigma, key, off)
    mu = L.forward_cache(actors[0], states.reshape(T * N, S))[2].reshape(T, N, -1)
    eps = (acts - mu) / np.float64(np.float32(sigma))
    R = L.returns(rewards)
    want = (R[None, :, None] * eps * (1 - mu ** 2)).sum((0, 1)) / N / np.float64(np.float32(sigma))
    np.testing.assert_allclose(g["b3"], want, rtol=1e-10)


def test_returns_sum_in_time_order():
    r = np.array([[1e16, 1.0], [1.0, 2.0], [-1e16, 3.0]])
    np.testing.assert_array_equal(L.returns(r), [((1e16 + 1.0) + -1e16), 6.0])


def _constant_agents(mus, S=4, H=3):
    """Agents whose weights are all zero and whose output biases are atanh(mu_k): each outputs the
    constant mean mu_k on every state (float64 parameters, so tanh(atanh(mu)) = mu to 1 ulp)."""
    out = []
    for mu in mus:
        mu = np.asarray(mu, np.float64)
        A = mu.size
        out.append({"W1": np.zeros((S, H)), "b1": np.zeros(H), "W2": np.zeros((H, H)), "b2": np.zeros(H),
                    "W3": np.zeros((H, A)), "b3": np.arctanh(mu)})
    return out


@pytest.mark.parametrize("i,want", [
    # Agent 0 at (0.5, -0.5) against (-0.25, 0.25) and (0.125, 0.0), lambda = 2, sigma = 0.5:
    # component 0: (0.5 + 0.25) + (0.5 - 0.125) = 1.125, times 1 - 0.25 = 0.75, over 0.25, times 2;
    # component 1: (-0.5 - 0.25) + (-0.5 - 0.0) = -1.25, same factors.
    (0, [6.75, -7.5]),
    # Agent 1 at (-0.25, 0.25): (-0.75 - 0.375, 0.75 + 0.25) times (1 - 0.0625) / 0.25 times 2.
    (1, [-8.4375, 7.5]),
    # Agent 2 at (0.125, 0.0): (-0.375 + 0.375, 0.5 - 0.25) times (1 - 0.015625, 1) / 0.25 times 2.
    (2, [0.0, 2.0]),
])
def test_diversity_gradient_closed_form(i, want):
    """Eq. (5) on its own (zero rewards, so eq. (4) drops out): agents with constant means mu_k.
    Ascending J + lambda sum_{j != i} KL(pi_j || pi_i), KL = |mu_j - mu_i|^2 / (2 sigma^2) averaged
    over the N T states, moves agent i's output bias by lambda sum_{j != i} (mu_i - mu_j) (1 - mu_i^2)
    / sigma^2: away from the other agents, and independent of N and T.  The expected values are
    worked by hand above; a flipped sign, a missing factor 2 or a lambda / N scale fails them."""
    agents = _constant_agents([[0.5, -0.5], [-0.25, 0.25], [0.125, 0.0]])
    for T, N in ((1, 1), (3, 5)):
        states = np.random.default_rng(T).standard_normal((T, N, 4)).astype(np.float32)
        g = L.policy_gradient(agents, i, states, np.zeros((T, N)), 0.5, 7, 0, 2.0)
        np.testing.assert_allclose(g["b3"], want, rtol=0, atol=1e-12)
        # Nothing else moves: every hidden activation is tanh(0) = 0 and every weight is zero.
        for name in ("W1", "b1", "W2", "b2", "W3"):
            assert np.abs(g[name]).max() == 0.0, name


def test_sampled_actions_follow_the_absolute_day():
    """Samples of a rollout that starts on a later day (resumed, or run in pieces): the pre-clip
    actions rebuilt for rows taken from day t0 on, clipped and rounded to float32, are exactly the
    actions the closed-loop oracle rollout drew on those days.  Keyed by the row index instead of
    the day, they are not."""
    from oracle.rollout import rollout_closed_loop
    from workload import EnvConfig, make_market
    D, T, N, t0, sigma, key = 4, 7, 6, 3, 0.3, 21
    cfg = EnvConfig(n_envs=N, n_stocks=D, n_ind=5, n_days=T)
    m = make_market(5, D, T)
    actors = make_actor_weights(ActorConfig(n_actors=2, in_dim=cfg.state_dim, hidden=8, out_dim=D, seed_base=70,
                                            bias_std=0.2))
    ro = rollout_closed_loop(cfg, m.close, m.ind, actors, T, sigma, key)
    states = ro["obs"][t0:T]  # the states acted on at days t0 .. T-1
    got = np.clip(L.sampled_actions(actors, states, sigma, key, 0, t0=t0), -1, 1).astype(np.float32)
    np.testing.assert_array_equal(got, ro["act"][t0:])
    wrong = np.clip(L.sampled_actions(actors, states, sigma, key, 0), -1, 1).astype(np.float32)
    assert not np.array_equal(wrong, ro["act"][t0:])
