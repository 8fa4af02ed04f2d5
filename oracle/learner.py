"""Oracle for the learner that consumes the rollout's samples (TEST INFRASTRUCTURE ONLY; see the
package docstring).

Section 4.1 writes the policy gradient as the Monte-Carlo estimate of eq. (4),
    grad J = (1/N) sum_n sum_t R(tau_n) grad log pi(a_t^n | s_t^n),
and Section 5.1 adds to an agent's objective the diversity term of eq. (5), lambda sum_{j != i}
KL(pi_j || pi_i) (the loss L_new = L - lambda sum KL, so the objective to ascend is J + lambda sum KL).
Readings:
  * agent i's policy is Gaussian, pi_i(a|s) = N(mu_i(s), sigma^2 I), with mu_i the actor network
    (tanh after every layer); the action sample is the one the rollout drew before clipping,
    a = abar(s) + sigma eps(n, t0 + t) with abar the ensemble mean and eps from the rollout's noise
    generator (key, global env index, absolute day; sample row t was drawn on day t0 + t);
  * R(tau_n) = sum_t r_t^n (gamma = 1, the stored rewards summed in t order);
  * the KL term is averaged over the N*T states: for equal sigma,
    KL(pi_j || pi_i) = |mu_j - mu_i|^2 / (2 sigma^2);
  * the gradient is taken at the float32 master weights; the sampled actions are data.
Everything is float64.  The gradient is written out by the chain rule through the three tanh
layers; `objective` is the scalar it differentiates, used by the finite-difference pins.
"""
from __future__ import annotations

import numpy as np

from .philox import noise
from .policy import actor_forward


def _f64(p):
    return {k: np.asarray(v, np.float64) for k, v in p.items()}


def forward_cache(p, x):
    """(X1, X2, mu) of one actor for rows x [n][S] (float64)."""
    p = _f64(p)
    x1 = np.tanh(np.asarray(x, np.float64) @ p["W1"] + p["b1"])
    x2 = np.tanh(x1 @ p["W2"] + p["b2"])
    mu = np.tanh(x2 @ p["W3"] + p["b3"])
    return x1, x2, mu


def sampled_actions(actors, states, sigma, noise_key, env_offset, mix=None, t0=0):
    """a = abar(s) + sigma eps for every (t, n), eps drawn on day t0 + t: float64 [T][N][A] (no
    clipping)."""
    T, N, S = states.shape
    rows = np.asarray(states, np.float64).reshape(T * N, S)
    K = len(actors)
    w = np.full(K, 1.0 / K) if mix is None else np.asarray(mix, np.float32).astype(np.float64)
    abar = None
    for k, p in enumerate(actors):
        term = w[k] * actor_forward(p, rows)
        abar = term if abar is None else abar + term
    A = abar.shape[1]
    eps = np.stack([noise(noise_key, env_offset + np.arange(N), t0 + t, A) for t in range(T)])
    return abar.reshape(T, N, A) + np.float64(np.float32(sigma)) * eps


def returns(rewards):
    """R(tau_n) = sum_t r_t^n, summed in ascending t: float64 [N]."""
    r = np.asarray(rewards, np.float64)
    acc = np.zeros(r.shape[1])
    for t in range(r.shape[0]):
        acc = acc + r[t]
    return acc


def objective(actors, i, states, actions, R, sigma, lam):
    """J_i = (1/N) sum_{n,t} R_n log pi_i(a|s) + lam/(N T) sum_{t,n} sum_{j != i} KL(pi_j || pi_i)."""
    T, N, S = states.shape
    rows = np.asarray(states, np.float64).reshape(T * N, S)
    s2 = np.float64(np.float32(sigma)) ** 2
    A = actions.shape[-1]
    mus = [forward_cache(p, rows)[2] for p in actors]
    a = np.asarray(actions, np.float64).reshape(T * N, A)
    Rr = np.repeat(np.asarray(R, np.float64)[None, :], T, axis=0).reshape(T * N)
    logp = -0.5 * ((a - mus[i]) ** 2).sum(1) / s2 - A * np.log(np.sqrt(2 * np.pi * s2))
    J = (Rr * logp).sum() / N
    kl = sum(((mus[j] - mus[i]) ** 2).sum() / (2 * s2) for j in range(len(actors)) if j != i)
    return J + lam * kl / (N * T)


def policy_gradient(actors, i, states, rewards, sigma, noise_key, env_offset, lam, mix=None, t0=0):
    """Gradient of `objective` with respect to actor i's parameters, with the actions the rollout
    sampled (row t on day t0 + t): dict W1, b1, W2, b2, W3, b3 (float64, the master weights'
    shapes)."""
    T, N, S = states.shape
    rows = np.asarray(states, np.float64).reshape(T * N, S)
    s2 = np.float64(np.float32(sigma)) ** 2
    acts = sampled_actions(actors, states, sigma, noise_key, env_offset, mix, t0)
    A = acts.shape[-1]
    a = acts.reshape(T * N, A)
    R = returns(rewards)
    Rr = np.repeat(R[None, :], T, axis=0).reshape(T * N)
    x1, x2, mu = forward_cache(actors[i], rows)
    # d objective / d mu_i per row.
    u = (Rr / N)[:, None] * (a - mu) / s2
    for j, p in enumerate(actors):
        if j != i:
            u = u + (lam / (N * T)) * (mu - forward_cache(p, rows)[2]) / s2
    p = _f64(actors[i])
    g3 = u * (1.0 - mu * mu)
    g2 = (g3 @ p["W3"].T) * (1.0 - x2 * x2)
    g1 = (g2 @ p["W2"].T) * (1.0 - x1 * x1)
    return {"W1": rows.T @ g1, "b1": g1.sum(0), "W2": x1.T @ g2, "b2": g2.sum(0), "W3": x2.T @ g3, "b3": g3.sum(0)}
