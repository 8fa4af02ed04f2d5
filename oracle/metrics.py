"""Backtest metrics and ensemble weights (TEST INFRASTRUCTURE ONLY; see the package docstring).

Section 6.1 evaluates trading agents with cumulative and annual return, annual volatility,
the Sharpe ratio of eq. (6), maximum drawdown, return over maximum drawdown (RoMaD), the
Sortino, Calmar and Omega ratios, and (Section 6.4) the win/loss ratio.  Section 5.2.1 weights
the stock ensemble by a softmax over the agents' validation Sharpe ratios after discarding
agents whose Sharpe ratio is too low; Section 5.2.2 combines the crypto ensemble by majority
vote.  Readings (the paper gives no formulas beyond eq. 6):
  * the equity curve of an environment is v_0 = initial asset, v_{t+1} = v_t + r_t / scale, and
    the period return is rho_t = v_{t+1} / v_t - 1;
  * annualisation uses P periods per year (252 for daily data): annual return
    (v_T / v_0)^(P/T) - 1, volatility std(rho) * sqrt(P) with the sample (n-1) deviation;
  * Sharpe = (mean(rho) - rf/P) / std(rho) * sqrt(P); Sortino uses the downside deviation
    sqrt(mean(min(rho - rf/P, 0)^2)) instead of std;
  * maximum drawdown = min_t (v_t / max_{s<=t} v_s - 1) <= 0; RoMaD = cumulative return /
    |maximum drawdown|; Calmar = annual return / |maximum drawdown|;
  * Omega with threshold 0 = sum(max(rho, 0)) / sum(max(-rho, 0)); win/loss = #(rho > 0) /
    #(rho < 0);
  * a ratio with a zero denominator follows IEEE division (inf or nan);
  * softmax weights: agents with Sharpe below a cut-off get weight 0, the rest get
    exp(s_k - max s) / sum; if every agent falls below the cut-off, the best one gets weight 1;
  * majority vote: the most frequent discrete action, ties to the lowest action index.
"""
from __future__ import annotations

import numpy as np

METRICS = ("cumulative_return", "annual_return", "annual_volatility", "sharpe", "max_drawdown",
           "romad", "sortino", "calmar", "omega", "win_loss")


def equity_curve(rewards, v0: float, reward_scale: float) -> np.ndarray:
    """v [T+1][N] from rewards [T][N]: v_{t+1} = v_t + r_t / scale (float64, in t order)."""
    r = np.asarray(rewards, dtype=np.float64)
    v = np.empty((r.shape[0] + 1,) + r.shape[1:], dtype=np.float64)
    v[0] = v0
    for t in range(r.shape[0]):
        v[t + 1] = v[t] + r[t] / reward_scale
    return v


def backtest_metrics(rewards, v0: float, reward_scale: float, periods_per_year: float = 252.0,
                     risk_free: float = 0.0) -> np.ndarray:
    """Metrics [N][10] in the order of METRICS."""
    v = equity_curve(rewards, v0, reward_scale)
    T = v.shape[0] - 1
    P = float(periods_per_year)
    rho = v[1:] / v[:-1] - 1.0
    excess = rho - risk_free / P
    with np.errstate(divide="ignore", invalid="ignore"):
        cum = v[-1] / v[0] - 1.0
        ann = (v[-1] / v[0]) ** (P / T) - 1.0
        sd = rho.std(axis=0, ddof=1) if T > 1 else np.full(rho.shape[1:], np.nan)
        vol = sd * np.sqrt(P)
        sharpe = excess.mean(axis=0) / sd * np.sqrt(P)
        peak = np.maximum.accumulate(v, axis=0)
        mdd = (v / peak - 1.0).min(axis=0)
        romad = cum / np.abs(mdd)
        down = np.sqrt(np.mean(np.minimum(excess, 0.0) ** 2, axis=0))
        sortino = excess.mean(axis=0) / down * np.sqrt(P)
        calmar = ann / np.abs(mdd)
        omega = np.maximum(rho, 0.0).sum(axis=0) / np.maximum(-rho, 0.0).sum(axis=0)
        winloss = (rho > 0).sum(axis=0) / (rho < 0).sum(axis=0)
    return np.stack([cum, ann, vol, sharpe, mdd, romad, sortino, calmar, omega, winloss], axis=-1)


def sharpe_softmax_weights(sharpe, min_sharpe: float = -np.inf) -> np.ndarray:
    """Softmax of the Sharpe ratios over agents at or above min_sharpe (float64 [K])."""
    s = np.asarray(sharpe, dtype=np.float64)
    keep = s >= min_sharpe
    if not keep.any():
        w = np.zeros_like(s)
        w[int(np.argmax(s))] = 1.0
        return w
    z = np.where(keep, s - s[keep].max(), -np.inf)
    e = np.where(keep, np.exp(z), 0.0)
    return e / e.sum()


def majority_vote(actions, n_actions: int) -> np.ndarray:
    """Most frequent discrete action over the agents (axis 0), ties to the lowest index."""
    a = np.asarray(actions)
    counts = np.stack([(a == j).sum(axis=0) for j in range(n_actions)], axis=-1)
    return np.argmax(counts, axis=-1)
