"""Pins for the oracle's noise generator and ensemble policy.

* Philox4x64-10 raw words are checked against numpy.random.Philox, a library
  implementation of the same published generator.  numpy advances its
  counter before producing a block, so block(c) equals numpy's output started
  at counter c - 1.
* The Gaussian map is checked by its moments and a Kolmogorov-Smirnov test.
* The ensemble rule of Section 5.2.1 (weighted average of the agents'
  actions) is checked on special cases with closed-form answers, and the
  float64 MLP against direct summation.
* bfloat16 rounding is checked against torch's float32 -> bfloat16 conversion.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle.env import orders
from oracle.philox import (box_muller, noise, noise_words, normals_from_words, philox4x64_10,
                           uniforms_from_words)
from oracle.policy import actor_forward, device_weights, ensemble_act, ensemble_mean, round_to_bf16
from workload import ActorConfig, make_actor_weights


def _numpy_block(counter, key):
    c = np.array(counter, dtype=np.uint64)
    # numpy increments before generating: start one below, borrowing across words.
    words = [int(x) for x in c]
    for i in range(4):
        if words[i] > 0:
            words[i] -= 1
            break
        words[i] = 2 ** 64 - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ([1, 0, 0, 0], [7, 0]),
    ([5, 17, 3, 0], [7, 0]),
    ([2047, 251, 7, 0], [123456789, 0]),
    ([0, 1, 0, 0], [7, 0]),                       # borrow across the first word
    ([0, 0, 0, 1], [2 ** 63 + 5, 2 ** 40]),       # borrow across three words, large key
    ([2 ** 64 - 1, 2 ** 64 - 1, 5, 9], [1, 2]),
])
def test_philox_matches_numpy(counter, key):
    ours = philox4x64_10(np.array(counter, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(ours, _numpy_block(counter, key))


def test_philox_vectorised_over_counters():
    rng = np.random.default_rng(0)
    ctr = rng.integers(1, 2 ** 62, size=(64, 4), dtype=np.uint64)
    key = np.array([99, 3], dtype=np.uint64)
    got = philox4x64_10(ctr, key)
    for i in range(64):
        assert np.array_equal(got[i], _numpy_block(ctr[i], key))


def test_uniform_map_exact_in_float32_and_open_interval():
    w = np.array([0, 1, 2 ** 41 - 1, 2 ** 41, 2 ** 64 - 1, 0x8000000000000000], dtype=np.uint64)
    u = uniforms_from_words(w)
    assert np.all(u > 0) and np.all(u < 1)
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 2.0 ** -24 and u[4] == 1.0 - 2.0 ** -24 and u[5] == 0.5 + 2.0 ** -24


def test_box_muller_closed_form():
    z0, z1 = box_muller(np.array([math.exp(-0.5)]), np.array([0.25]))
    assert abs(z0[0]) < 1e-15 and abs(z1[0] - 1.0) < 1e-15
    z0, z1 = box_muller(np.array([math.exp(-2.0)]), np.array([0.5]))
    assert abs(z0[0] + 2.0) < 1e-15 and abs(z1[0]) < 1e-15


def test_normals_moments_and_ks():
    n = 250_000
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n, dtype=np.uint64)
    z = normals_from_words(philox4x64_10(ctr, np.array([7, 0], dtype=np.uint64))).ravel()
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_noise_layout():
    eps = noise(7, np.arange(3, 6), 11, 30)
    assert eps.shape == (3, 30)
    w = noise_words(7, np.arange(3, 6), 11, 30)
    assert w.shape == (3, 8, 4)
    direct = philox4x64_10(np.array([4, 11, 5, 0], dtype=np.uint64), np.array([7, 0], dtype=np.uint64))
    assert np.array_equal(w[1, 5], direct)
    assert np.array_equal(eps[1, 20:24], normals_from_words(direct))


def _tiny_cfg(K=2, S=5, H=4, A=3, bias=0.3):
    return ActorConfig(n_actors=K, in_dim=S, hidden=H, out_dim=A, bias_std=bias)


def test_mlp_matches_direct_summation():
    cfg = _tiny_cfg()
    actors = make_actor_weights(cfg)
    obs = np.random.default_rng(1).standard_normal((3, cfg.in_dim)).astype(np.float32)
    p = actors[0]
    for n in range(3):
        x = [float(v) for v in obs[n]]
        for W, b in ((p["W1"], p["b1"]), (p["W2"], p["b2"]), (p["W3"], p["b3"])):
            x = [math.tanh(math.fsum(x[i] * float(W[i, j]) for i in range(len(x))) + float(b[j]))
                 for j in range(W.shape[1])]
        assert np.allclose(actor_forward(p, obs[n:n + 1])[0], x, rtol=0, atol=1e-14)


def test_zero_weights_give_tanh_of_output_bias():
    cfg = _tiny_cfg(K=1)
    p = make_actor_weights(cfg)[0]
    for name in ("W1", "W2", "W3"):
        p[name] = np.zeros_like(p[name])
    obs = np.ones((2, cfg.in_dim), np.float32)
    assert np.array_equal(actor_forward(p, obs), np.broadcast_to(np.tanh(p["b3"].astype(np.float64)), (2, 3)))


def test_two_actor_average_closed_form():
    """b3 = atanh(0.5) for one actor and atanh(-0.25) for the other, equal weights: a_bar = 0.125, q = 12."""
    cfg = _tiny_cfg(K=2, bias=0.0)
    actors = make_actor_weights(cfg)
    for p, v in zip(actors, (0.5, -0.25)):
        p["W3"] = np.zeros_like(p["W3"])
        p["b3"] = np.full(cfg.out_dim, np.arctanh(v), np.float32)
    obs = np.random.default_rng(2).standard_normal((4, cfg.in_dim)).astype(np.float32)
    mean = ensemble_mean(actors, obs)
    assert np.allclose(mean, 0.125, atol=1e-7)
    a = ensemble_act(actors, obs, 0, 0, 0.0, 7)
    assert np.all(orders(a, 100) == 12)


def test_single_actor_and_one_hot_weights_reproduce_that_actor():
    cfg = _tiny_cfg(K=3)
    actors = make_actor_weights(cfg)
    obs = np.random.default_rng(3).standard_normal((5, cfg.in_dim)).astype(np.float32)
    for k in range(3):
        mix = np.zeros(3, np.float32)
        mix[k] = 1.0
        assert np.array_equal(ensemble_mean(actors, obs, mix), actor_forward(actors[k], obs))
    assert np.array_equal(ensemble_mean(actors[:1], obs), actor_forward(actors[0], obs))


def test_noise_added_after_average_then_clipped():
    cfg = _tiny_cfg(K=2, A=30)
    actors = make_actor_weights(cfg)
    obs = np.random.default_rng(4).standard_normal((6, cfg.in_dim)).astype(np.float32)
    a, mean = ensemble_act(actors, obs, 5, 100, 0.1, 7, return_mean=True)
    eps = noise(7, np.arange(100, 106), 5, 30)
    assert np.array_equal(a, np.clip(mean + np.float64(np.float32(0.1)) * eps, -1, 1).astype(np.float32))
    big, mean = ensemble_act(actors, obs, 5, 100, 50.0, 7, return_mean=True)
    pre = mean + 50.0 * eps
    assert np.all(np.abs(big) <= 1.0)
    assert np.array_equal(big[np.abs(pre) > 1], np.sign(pre[np.abs(pre) > 1]).astype(np.float32))
    assert (np.abs(pre) > 1).mean() > 0.9


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([
        rng.standard_normal(10000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.3895314e38, 1e-40, -1e-42], np.float32),
        # exact ties: bit 15 set and lower bits zero, both parities of the kept lsb
        np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x3F80C000], dtype=np.uint32).view(np.float32),
    ])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(round_to_bf16(x).view(np.uint32), ref.view(np.uint32))


def test_device_weights_bf16_rounds_matrices_only():
    cfg = _tiny_cfg(K=1, bias=0.3)
    p = make_actor_weights(cfg)[0]
    q = device_weights([p], "bf16")[0]
    assert np.array_equal(q["b1"], p["b1"])
    assert np.array_equal(q["W2"], round_to_bf16(p["W2"]))
    assert not np.array_equal(q["W2"], p["W2"])
