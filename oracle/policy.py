"""Oracle ensemble policy (TEST INFRASTRUCTURE ONLY; see the package docstring).

The stock-trading ensemble of Section 5.2.1 acts on the weighted average of
its agents' actions.  Each agent's policy (Section 3.1, Policy) is a
deterministic MLP mean mu_k(s) = tanh(W3 tanh(W2 tanh(W1 s + b1) + b2) + b3)
(row-vector convention: x @ W).  Readings:
  * the average is over the actors' means, a_bar = sum_k w_k mu_k with
    w_k = 1/K unless weights are given (the softmax-of-Sharpe weights of
    Section 5.2.1 are passed in the same way);
  * exploration noise is added after averaging, a = clip(a_bar + sigma*eps,
    -1, 1), eps from the counter-based generator in philox.py;
  * for the bfloat16 path the oracle evaluates, in float64, the weight
    matrices rounded to bfloat16 exactly as the device stores them (biases
    stay float32), so the comparison measures arithmetic error only.
Everything is float64; the returned action is rounded to float32 once.
"""
from __future__ import annotations

import numpy as np

from .philox import noise


def round_to_bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returned as float32.

    bfloat16 keeps the top 16 bits of the float32 encoding.  Rounding adds
    0x7FFF plus the lowest kept bit before truncating, which is round to
    nearest, ties to even.  NaN stays NaN.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (rounded & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), x, out).astype(np.float32)


def actor_forward(p, obs) -> np.ndarray:
    """mu = tanh(tanh(tanh(obs W1 + b1) W2 + b2) W3 + b3) in float64; obs [n][S] -> [n][A]."""
    x = np.asarray(obs, dtype=np.float64)
    x = np.tanh(x @ np.asarray(p["W1"], np.float64) + np.asarray(p["b1"], np.float64))
    x = np.tanh(x @ np.asarray(p["W2"], np.float64) + np.asarray(p["b2"], np.float64))
    return np.tanh(x @ np.asarray(p["W3"], np.float64) + np.asarray(p["b3"], np.float64))


def device_weights(actors, dtype: str):
    """The weights as the device computes with them: float32, or W matrices rounded to bf16."""
    if dtype == "f32":
        return actors
    if dtype != "bf16":
        raise ValueError(dtype)
    out = []
    for p in actors:
        q = dict(p)
        for name in ("W1", "W2", "W3"):
            q[name] = round_to_bf16(p[name])
        out.append(q)
    return out


def ensemble_mean(actors, obs, mix=None) -> np.ndarray:
    """a_bar = sum_k w_k mu_k, summed in ascending k (float64 [n][A])."""
    K = len(actors)
    w = np.full(K, 1.0 / K) if mix is None else np.asarray(mix, dtype=np.float32).astype(np.float64)
    acc = None
    for k, p in enumerate(actors):
        term = w[k] * actor_forward(p, obs)
        acc = term if acc is None else acc + term
    return acc


def ensemble_act(actors, obs, t: int, env_offset: int, sigma: float, noise_key: int, mix=None,
                 return_mean: bool = False, env_ids=None):
    """a = fl32(clip(a_bar + sigma*eps(n, t, d), -1, 1)).

    Row i of obs is environment env_offset + i, or env_ids[i] when env_ids is given.
    """
    mean = ensemble_mean(actors, obs, mix)
    sig = np.float64(np.float32(sigma))
    if sig != 0.0:
        ids = np.arange(env_offset, env_offset + mean.shape[0]) if env_ids is None else np.asarray(env_ids)
        eps = noise(noise_key, ids, t, mean.shape[1])
        pre = mean + sig * eps
    else:
        pre = mean
    act = np.clip(pre, -1.0, 1.0).astype(np.float32)
    return (act, mean) if return_mean else act
