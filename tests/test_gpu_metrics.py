"""GPU backtest metrics against the oracle's (1e-10 relative; inf and NaN must match)."""
import numpy as np
import pytest

from _helpers import cuda, env_case
from oracle.metrics import backtest_metrics
from oracle.rollout import rollout_driven
from workload import make_actions

pytestmark = pytest.mark.gpu


def _close(got, want):
    both_nan = np.isnan(got) & np.isnan(want)
    same_inf = np.isinf(got) & np.isinf(want) & (np.sign(got) == np.sign(want))
    fin = np.isfinite(want)
    with np.errstate(invalid="ignore"):  # inf - inf where both are infinite; judged by same_inf
        near = np.abs(got - want) <= 1e-10 * np.maximum(np.abs(want), 1e-300)
    ok = both_nan | same_inf | (fin & near)
    return ok


@pytest.mark.parametrize("N,T,rf", [(37, 60, 0.0), (300, 252, 0.02), (5, 2, 0.0)])
def test_metrics_match_oracle(N, T, rf):
    import torch
    from paper_2501_10709_amd import binding as B
    dev = cuda()
    cfg, m = env_case(N, 30, 5, T, 90 + N)
    acts = make_actions(91, T, N, 30)
    ref = rollout_driven(cfg, m.close, m.ind, acts)
    rew = torch.from_numpy(ref["reward"]).to(dev)
    got = B.fm_backtest_metrics(rew, cfg.init_cash, cfg.reward_scale, 252.0, rf).cpu().numpy()
    want = backtest_metrics(ref["reward"], cfg.init_cash, cfg.reward_scale, 252.0, rf)
    ok = _close(got, want)
    assert ok.all(), (np.argwhere(~ok)[:5], got[~ok][:5], want[~ok][:5])


def test_metrics_special_cases_and_per_env_start():
    import torch
    from paper_2501_10709_amd import binding as B
    dev = cuda()
    v = np.array([1024.0 * 1.5 ** t for t in range(11)])
    r = np.stack([(v[1:] - v[:-1]) * 2.0 ** -12, -(v[1:] - v[:-1]) * 2.0 ** -20], axis=1)  # [T][2]
    v0 = np.array([1024.0, 4096.0])
    got = B.fm_backtest_metrics(torch.from_numpy(r).to(dev), 0.0, 2.0 ** -12,
                                d_init_asset=torch.from_numpy(v0).to(dev)).cpu().numpy()
    want = np.stack([backtest_metrics(r[:, :1], 1024.0, 2.0 ** -12)[0], backtest_metrics(r[:, 1:], 4096.0, 2.0 ** -12)[0]])
    assert _close(got, want).all()
    assert got[0, 3] == np.inf and got[0, 4] == 0.0
