"""The GPU chain's partial fill (a buy whose whole order does not fit) starts from the estimate
k = floor(cash * rc1), rc1 a Newton-refined hardware reciprocal of the one-share debit, keeps it
when the debits of k and k+1 bracket cash and otherwise takes unit steps.  This mirrors that
arithmetic on the host with the reciprocal's seed error pushed to the hardware bound (2^-23
relative, either sign), and checks on random and adversarial cases (cash within a few ulp of a
debit) that the result equals the exhaustive definition and that at most one step is taken."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.env import buy_quantity

ONE_P = float(np.float64(1.0) + np.float64(1e-3))


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))  # exact product and sum, one rounding


def _fill(cash, p, q, seed_err):
    c1 = p * ONE_P
    r = (1.0 / c1) * (1.0 + seed_err)              # worst-case hardware seed
    r = _fma(_fma(-c1, r, 1.0), r, r)              # one Newton step, as on the device
    qm1 = float(q - 1)
    kd = max(min(np.floor(cash * r), qm1), 0.0)
    debit = lambda k: (p * float(k)) * ONE_P
    k, steps = int(kd), 0
    dk = debit(kd) if kd > 0 else 0.0
    if not dk <= cash or (kd < qm1 and debit(kd + 1) <= cash):
        while k + 1 < q and debit(k + 1) <= cash:
            k, steps = k + 1, steps + 1
        while k > 0 and not debit(k) <= cash:
            k, steps = k - 1, steps + 1
    return k, steps


def _cases(rng, n, qmax=100):
    out = []
    for _ in range(n):
        p = float(np.float32(rng.uniform(0.5, 3000.0)))
        q = int(rng.integers(2, qmax + 1))
        k = int(rng.integers(1, q))
        base = (p * k) * ONE_P
        if rng.integers(0, 4) == 0:
            cash = float(rng.uniform(p * ONE_P, (p * q) * ONE_P))
        else:
            cash = base
            for _ in range(int(rng.integers(0, 5))):
                cash = float(np.nextafter(cash, np.inf if rng.random() < 0.5 else -np.inf))
        if p * ONE_P <= cash < (p * q) * ONE_P:
            out.append((cash, p, q))
    return out


@pytest.mark.parametrize("seed_err", [0.0, 2.0**-23, -(2.0**-23), 0.7 * 2.0**-23])
def test_estimate_and_steps_are_exact(seed_err):
    cases = _cases(np.random.default_rng(123), 3000)
    assert len(cases) > 2000
    for cash, p, q in cases:
        k, steps = _fill(cash, p, q, seed_err)
        want = int(buy_quantity(np.array([cash]), np.float32(p), np.array([q]), ONE_P)[0])
        assert k == want and steps <= 1, (cash, p, q, k, want, steps)


def test_orders_near_the_configuration_bound():
    # hmax up to 2^20: quotients up to 2^20 keep the estimate within one share.
    rng = np.random.default_rng(7)
    for _ in range(300):
        p = float(np.float32(rng.uniform(0.01, 2.0)))
        q = int(rng.integers(2**19, 2**20))
        k = int(rng.integers(1, q))
        cash = float(np.nextafter((p * k) * ONE_P, -np.inf if rng.random() < 0.5 else np.inf))
        if not (p * ONE_P <= cash < (p * q) * ONE_P):
            continue
        for seed_err in (2.0**-23, -(2.0**-23)):
            kk, steps = _fill(cash, p, q, seed_err)
            assert steps <= 1
            assert (p * kk) * ONE_P <= cash < (p * (kk + 1)) * ONE_P
