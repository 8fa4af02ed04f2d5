"""Pins for the oracle's backtest metrics, Sharpe-softmax weights and majority vote.

Expected values come from closed forms on constructed equity curves (exact in binary), from a
hand-worked drawdown example, and from Python's statistics module (a library routine) for the
sample mean and deviation.
"""
import math
import statistics
from fractions import Fraction

import numpy as np

from oracle.metrics import (METRICS, backtest_metrics, equity_curve, majority_vote,
                            sharpe_softmax_weights)

IDX = {name: i for i, name in enumerate(METRICS)}


def _rewards_from_curve(v, scale):
    v = np.asarray(v, dtype=np.float64)
    return ((v[1:] - v[:-1]) * scale)[:, None]


def test_geometric_curve_closed_forms():
    """v_t = 1024 * 1.5^t is exact in float64: every return is 0.5, no deviation, no drawdown."""
    v = [1024.0 * 1.5 ** t for t in range(11)]
    r = _rewards_from_curve(v, 2.0 ** -12)
    assert np.array_equal(equity_curve(r, 1024.0, 2.0 ** -12)[:, 0], v)
    m = backtest_metrics(r, 1024.0, 2.0 ** -12, 252.0)[0]
    assert m[IDX["cumulative_return"]] == 1.5 ** 10 - 1
    assert math.isclose(m[IDX["annual_return"]], 1.5 ** 252 - 1, rel_tol=1e-12)
    assert m[IDX["annual_volatility"]] == 0.0
    assert m[IDX["max_drawdown"]] == 0.0
    for name in ("sharpe", "sortino", "romad", "calmar", "omega", "win_loss"):
        assert m[IDX[name]] == np.inf, name


def test_hand_worked_drawdown_and_ratios():
    v = [100.0, 120.0, 90.0, 130.0, 65.0, 80.0]
    r = _rewards_from_curve(v, 1.0)
    m = backtest_metrics(r, 100.0, 1.0, 252.0)[0]
    rho = [Fraction(v[i + 1]) / Fraction(v[i]) - 1 for i in range(5)]
    assert math.isclose(m[IDX["cumulative_return"]], -0.2, rel_tol=1e-15)  # 80/100 - 1
    assert m[IDX["max_drawdown"]] == -0.5             # 65 after the 130 peak
    assert m[IDX["win_loss"]] == 1.5                  # 3 gains, 2 losses
    omega = sum(x for x in rho if x > 0) / -sum(x for x in rho if x < 0)
    assert math.isclose(m[IDX["omega"]], float(omega), rel_tol=1e-14)
    rf = [float(x) for x in rho]
    sd = statistics.stdev(rf)
    assert math.isclose(m[IDX["annual_volatility"]], sd * math.sqrt(252), rel_tol=1e-12)
    assert math.isclose(m[IDX["sharpe"]], statistics.mean(rf) / sd * math.sqrt(252), rel_tol=1e-12)
    down = math.sqrt(sum(min(x, 0.0) ** 2 for x in rf) / 5)
    assert math.isclose(m[IDX["sortino"]], statistics.mean(rf) / down * math.sqrt(252), rel_tol=1e-12)
    assert math.isclose(m[IDX["romad"]], -0.2 / 0.5, rel_tol=1e-14)
    assert math.isclose(m[IDX["cumulative_return"]] / 0.5, m[IDX["romad"]], rel_tol=1e-15)
    ann = (0.8) ** (252 / 5) - 1
    assert math.isclose(m[IDX["annual_return"]], ann, rel_tol=1e-12)
    assert math.isclose(m[IDX["calmar"]], ann / 0.5, rel_tol=1e-12)


def test_risk_free_shifts_sharpe_only():
    rng = np.random.default_rng(0)
    r = rng.normal(5.0, 40.0, size=(60, 3))
    a = backtest_metrics(r, 1e6, 2.0 ** -12, 252.0, 0.0)
    b = backtest_metrics(r, 1e6, 2.0 ** -12, 252.0, 0.05)
    assert np.array_equal(a[:, IDX["annual_volatility"]], b[:, IDX["annual_volatility"]])
    assert np.all(b[:, IDX["sharpe"]] < a[:, IDX["sharpe"]])
    # Sharpe = (mean - rf/P) / sd * sqrt(P): the shift times the annual volatility is rf.
    shift = (a[:, IDX["sharpe"]] - b[:, IDX["sharpe"]]) * a[:, IDX["annual_volatility"]]
    assert np.allclose(shift, 0.05, rtol=1e-9)


def test_softmax_weights():
    assert np.allclose(sharpe_softmax_weights([0.7, 0.7, 0.7]), [1 / 3] * 3, atol=0, rtol=1e-15)
    w = sharpe_softmax_weights([1.0, 2.0, 0.5])
    assert math.isclose(w[1] / w[0], math.e, rel_tol=1e-14)
    assert math.isclose(w.sum(), 1.0, rel_tol=1e-15)
    w = sharpe_softmax_weights([1.0, -0.5, 2.0], min_sharpe=0.0)
    assert w[1] == 0.0 and math.isclose(w[2] / w[0], math.e, rel_tol=1e-14)
    w = sharpe_softmax_weights([-1.0, -0.2, -3.0], min_sharpe=0.0)
    assert list(w) == [0.0, 1.0, 0.0]


def test_majority_vote():
    acts = np.array([[0, 2, 1, 1], [2, 2, 0, 1], [2, 1, 2, 0]])  # 3 agents x 4 samples
    assert list(majority_vote(acts, 3)) == [2, 2, 0, 1]      # sample 2 is a 3-way tie -> lowest
    assert list(majority_vote(np.array([[1, 0], [0, 1]]), 2)) == [0, 0]
