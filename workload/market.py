"""Seeded synthetic daily market: GBM closes, derived OHLCV and five indicators.

Stand-in for the paper's daily OHLCV of the 30 Dow Jones stocks (Section 6.1).
The state of the MDP carries prices p_t and an indicator vector f_t of I values
per stock (Section 3.1); the paper names MACD first among its indicators
(Sections 3.1 and 6.1).  Five indicators are produced, in this order:

  0  MA5 / close - 1
  1  MA20 / close - 1
  2  RSI14 (Wilder smoothing) / 100 - 0.5
  3  volume / MA20(volume) - 1
  4  MACD / close, MACD = EMA12 - EMA26

Generation runs in float64 on the host and the arrays handed to either side
are float32.  Nothing here is part of the environment's step arithmetic.
"""
from __future__ import annotations

import dataclasses

import numpy as np

BURN_IN = 40  # days generated before day 0 so every indicator has its full window


@dataclasses.dataclass
class Market:
    close: np.ndarray   # float32 [T+1][D]
    ind: np.ndarray     # float32 [T+1][I][D], indicator-major inside a day
    open: np.ndarray    # float32 [T+1][D]
    high: np.ndarray    # float32 [T+1][D]
    low: np.ndarray     # float32 [T+1][D]
    volume: np.ndarray  # float32 [T+1][D]

    @property
    def n_days(self) -> int:
        return self.close.shape[0] - 1

    @property
    def n_stocks(self) -> int:
        return self.close.shape[1]

    @property
    def n_ind(self) -> int:
        return self.ind.shape[1]


def gbm_closes(rng: np.random.Generator, n_steps: int, n_stocks: int, drift: float, vol,
               s0_lo: float = 50.0, s0_hi: float = 300.0) -> np.ndarray:
    """S_{t+1} = S_t exp(mu - vol^2/2 + vol Z), S_0 ~ U[s0_lo, s0_hi]; float64 [n_steps+1][D]."""
    vol = np.broadcast_to(np.asarray(vol, dtype=np.float64), (n_stocks,))
    s0 = rng.uniform(s0_lo, s0_hi, size=n_stocks)
    z = rng.standard_normal((n_steps, n_stocks))
    logret = (drift - 0.5 * vol * vol) + vol * z
    logs = np.concatenate([np.log(s0)[None, :], np.log(s0)[None, :] + np.cumsum(logret, axis=0)], axis=0)
    return np.exp(logs)


def _rolling_mean(x: np.ndarray, w: int) -> np.ndarray:
    """Trailing mean over the last w rows (fewer at the start), axis 0."""
    c = np.cumsum(np.concatenate([np.zeros((1,) + x.shape[1:]), x], axis=0), axis=0)
    out = np.empty_like(x)
    for t in range(x.shape[0]):
        lo = max(0, t + 1 - w)
        out[t] = (c[t + 1] - c[lo]) / (t + 1 - lo)
    return out


def _ema(x: np.ndarray, span: int) -> np.ndarray:
    alpha = 2.0 / (span + 1.0)
    out = np.empty_like(x)
    out[0] = x[0]
    for t in range(1, x.shape[0]):
        out[t] = alpha * x[t] + (1.0 - alpha) * out[t - 1]
    return out


def _rsi_wilder(close: np.ndarray, n: int = 14) -> np.ndarray:
    """Wilder's RSI in [0, 100]; rows before the first full window use the running mean."""
    delta = np.diff(close, axis=0, prepend=close[:1])
    gain = np.maximum(delta, 0.0)
    loss = np.maximum(-delta, 0.0)
    ag = np.empty_like(close)
    al = np.empty_like(close)
    ag[0], al[0] = gain[0], loss[0]
    for t in range(1, close.shape[0]):
        k = min(t, n)  # simple running mean until n samples exist, then Wilder smoothing
        ag[t] = (ag[t - 1] * (k - 1) + gain[t]) / k
        al[t] = (al[t - 1] * (k - 1) + loss[t]) / k
    with np.errstate(divide="ignore", invalid="ignore"):
        rs = np.where(al > 0, ag / np.where(al > 0, al, 1.0), np.inf)
        rsi = np.where(np.isinf(rs), 100.0, 100.0 - 100.0 / (1.0 + rs))
    rsi = np.where((ag == 0) & (al == 0), 50.0, rsi)
    return rsi


def make_market(seed: int, n_stocks: int, n_days: int, n_ind: int = 5, drift: float = 3e-4,
                vol=0.02) -> Market:
    """Seeded market of n_days+1 daily rows for n_stocks stocks (numpy PCG64)."""
    if not 0 <= n_ind <= 5:
        raise ValueError("n_ind must be in 0..5")
    rng = np.random.default_rng(seed)
    n_total = n_days + BURN_IN
    close = gbm_closes(rng, n_total, n_stocks, drift, vol)
    volv = np.broadcast_to(np.asarray(vol, dtype=np.float64), (n_stocks,))
    z = rng.standard_normal((4, n_total + 1, n_stocks))
    prev = np.concatenate([close[:1], close[:-1]], axis=0)
    open_ = prev * np.exp(0.2 * volv * z[0])
    high = np.maximum(open_, close) * (1.0 + np.abs(0.5 * volv * z[1]))
    low = np.minimum(open_, close) * (1.0 - np.abs(0.5 * volv * z[2]))
    vbase = rng.uniform(1e6, 1e7, size=n_stocks)
    volume = vbase * np.exp(0.3 * z[3])

    feats = [
        _rolling_mean(close, 5) / close - 1.0,
        _rolling_mean(close, 20) / close - 1.0,
        _rsi_wilder(close) / 100.0 - 0.5,
        volume / _rolling_mean(volume, 20) - 1.0,
        (_ema(close, 12) - _ema(close, 26)) / close,
    ][:n_ind]
    ind = np.stack(feats, axis=1) if feats else np.zeros((n_total + 1, 0, n_stocks))  # [rows][I][D]
    sl = slice(BURN_IN, BURN_IN + n_days + 1)
    f32 = lambda a: np.ascontiguousarray(a[sl], dtype=np.float32)
    return Market(close=f32(close), ind=f32(ind), open=f32(open_), high=f32(high), low=f32(low),
                  volume=f32(volume))
