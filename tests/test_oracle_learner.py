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
