"""Brute force over every order sequence of a 2-stock, 3-day market.

With hmax = 3 each day has 7 x 7 order pairs, so three days give 49^3 =
117,649 sequences; each sequence is one environment of the vectorised oracle.
An independent reference recomputes every sequence with exact integer
arithmetic (money counted in units of 2^-12) and finds each buy by trying
every k from q down to 0.  With cost rate 2^-10 and prices that are
multiples of 1/4 every float64 operation of the oracle is exact, so the two
must agree bit for bit.  With the float64 cost rate 1e-3 the reference uses
the float64 constants fl(1-c), fl(1+c) in exact rational arithmetic; holdings
may then differ only where a debit lies within rounding of the cash, and such
cases are counted and must be rare.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle.env import OracleEnv
from workload import EnvConfig

HMAX = 3
QS = list(range(-HMAX, HMAX + 1))
UNIT = 2 ** 12


def _all_sequences():
    pairs = list(itertools.product(QS, QS))
    seqs = np.array(list(itertools.product(pairs, repeat=3)), dtype=np.int32)  # [49^3][3][2]
    return seqs


def _actions_for(q):
    """float32 actions whose float32 product with hmax truncates to exactly q."""
    a = (q + 0.25 * np.sign(q)) / HMAX
    return np.clip(a, -1.0, 1.0).astype(np.float32)


def _reference_int(prices, cash0, seqs):
    """Exact reference, money in units of 2^-12, cost rate 2^-10."""
    P = [[int(Fraction(float(p)) * UNIT) for p in row] for row in prices]
    out_cash, out_hold, out_rew = [], [], []
    for seq in seqs.tolist():
        cash = int(cash0 * UNIT)
        h = [0, 0]
        v = cash
        rews = []
        for t, q in enumerate(seq):
            p = P[t]
            for d in range(2):
                if q[d] < 0:
                    s = min(h[d], -q[d])
                    cash += p[d] * s - (p[d] * s) // 1024     # p*s*(1 - 2^-10); divisible by 1024
                    h[d] -= s
            for d in range(2):
                if q[d] > 0:
                    k = q[d]
                    while k > 0 and p[d] * k + (p[d] * k) // 1024 > cash:
                        k -= 1
                    cash -= p[d] * k + (p[d] * k) // 1024
                    h[d] += k
            v_new = cash + P[t + 1][0] * h[0] + P[t + 1][1] * h[1]
            rews.append(v_new - v)
            v = v_new
        out_cash.append(cash)
        out_hold.append(h)
        out_rew.append(rews)
    return np.array(out_cash, dtype=object), np.array(out_hold), np.array(out_rew, dtype=object)


def _oracle(prices, cash0, seqs, cost_rate):
    close = np.array(prices, dtype=np.float32)
    cfg = EnvConfig(n_envs=seqs.shape[0], n_stocks=2, n_ind=1, n_days=3, hmax=HMAX, cost_rate=cost_rate,
                    init_cash=cash0, reward_scale=1.0)
    env = OracleEnv(cfg, close, np.zeros((4, 1, 2), np.float32))
    rews = []
    for t in range(3):
        _, r, _, _ = env.step(_actions_for(seqs[:, t, :]))
        rews.append(r)
    return env, np.stack(rews, axis=1)


MARKETS = [
    ([[100.0, 50.0], [104.0, 48.0], [96.5, 52.25], [101.0, 49.5]], 300.0),
    ([[37.5, 12.25], [36.0, 13.0], [40.75, 11.5], [39.0, 12.0]], 120.0),
]


@pytest.mark.parametrize("prices,cash0", MARKETS)
def test_bruteforce_exact_cost(prices, cash0):
    seqs = _all_sequences()
    env, rew = _oracle(prices, cash0, seqs, cost_rate=2.0 ** -10)
    ref_cash, ref_hold, ref_rew = _reference_int(prices, cash0, seqs)
    assert np.array_equal(env.hold, ref_hold)
    assert all(float(Fraction(c, UNIT)) == x for c, x in zip(ref_cash, env.cash))
    for t in range(3):
        assert all(float(Fraction(int(r), UNIT)) == x for r, x in zip(ref_rew[:, t], rew[:, t]))


def test_bruteforce_float_cost_rate():
    """c = 1e-3: exact rational arithmetic on the float64 constants; holdings agree except at ties."""
    prices, cash0 = MARKETS[0]
    seqs = _all_sequences()
    env, _ = _oracle(prices, cash0, seqs, cost_rate=1e-3)
    one_m = Fraction(1.0 - 1e-3)
    one_p = Fraction(1.0 + 1e-3)
    P = [[Fraction(float(np.float32(p))) for p in row] for row in prices]
    sample = np.random.default_rng(0).choice(seqs.shape[0], 4000, replace=False)
    mismatches = 0
    for i in sample:
        cash = Fraction(cash0)
        h = [0, 0]
        close_call = False
        for t in range(3):
            q = seqs[i, t]
            for d in range(2):
                if q[d] < 0:
                    s = min(h[d], -int(q[d]))
                    cash += P[t][d] * s * one_m
                    h[d] -= s
            for d in range(2):
                if q[d] > 0:
                    k = int(q[d])
                    while k > 0 and P[t][d] * k * one_p > cash:
                        k -= 1
                    for kk in (k, k + 1):
                        if abs(P[t][d] * kk * one_p - cash) <= Fraction(1, 2 ** 40):
                            close_call = True
                    cash -= P[t][d] * k * one_p
                    h[d] += k
        if list(env.hold[i]) != h:
            assert close_call, (i, seqs[i].tolist(), env.hold[i], h)
            mismatches += 1
        else:
            assert abs(float(cash) - env.cash[i]) <= 1e-12 * max(1.0, abs(float(cash)))
    assert mismatches <= len(sample) // 100
