"""The crypto serving path on the GPU (through include/crypto_serve.h) against the oracle.

Parity: the oracle is driven by the actions the GPU chose, evaluating the agents (bfloat16-rounded
weights, float64 arithmetic) on the states it reaches.  Positions and trade counts must match
exactly; cash, values and the running statistics within 1e-12 relative; the averaged
probabilities within 2e-2 absolute; every explored action exactly; every greedy action wherever
the oracle's decision has a margin above twice that tolerance.  Batch invariance: a request's
results are bit-identical alone, in a mix of requests, and under another chunk length.
"""
import numpy as np
import pytest

from oracle import crypto as oc
from oracle.policy import device_weights
from workload import pack_actor_weights
from workload.crypto import crypto_actors, make_crypto_agents, make_ticks

from _helpers import TOL_BF16, TOL_F64_REL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def market():
    return make_ticks(seed=21, n_ticks=20_000)


def _server(market, K=5, rule=0, eps=0.05, rows=64, chunk=100, **kw):
    from paper_2501_10709_amd.serve import CryptoServer
    actors = make_crypto_agents(crypto_actors(n_actors=K))
    srv = CryptoServer(market.mid, market.feat, pack_actor_weights(actors), K, rule=rule, eps=eps, tile_rows=rows,
                       chunk_ticks=chunk, **kw)
    return srv, actors


def _check_request(market, actors, q, res, act, prob, rule, eps, fee=2e-4):
    K = len(actors)
    dev = device_weights(actors, "bf16")
    obs = []
    st, probs, chosen, greedy, explored, _ = oc.rollout(
        market, dev, q["n"], q["T"], q["start"], q["stride"], q["key"], eps, fee=fee, mode=rule, actions=act,
        obs_out=obs)
    assert (res["ticks"] == q["T"]).all()
    assert (res["position"] == st["pos"]).all()
    assert (res["trades"] == st["trades"]).all()
    for name, key in [("cash", "cash"), ("value", "value"), ("sum_r", "sum_r"), ("sum_r2", "sum_r2"),
                      ("peak", "peak"), ("max_drawdown", "mdd")]:
        scale = np.maximum(np.abs(st[key]), np.abs(st["value"]) if key in ("sum_r", "max_drawdown") else 1.0)
        err = np.abs(res[name] - st[key])
        assert (err <= TOL_F64_REL * np.maximum(scale, 1.0)).all(), (name, err.max())
    # Exploration draws decide exactly.
    rand = np.stack([oc.exploration(q["key"], np.arange(q["n"]), t, eps)[1] for t in range(q["T"])])
    assert (act[explored] == rand[explored]).all()
    x = np.stack(obs)                                            # [T][n][16]
    if rule == oc.AVG_SOFTMAX:
        assert np.abs(prob - probs).max() <= TOL_BF16
        srt = np.sort(probs, axis=-1)
        safe = (~explored) & (srt[..., 2] - srt[..., 1] > 2 * TOL_BF16)
        assert (act[safe] == greedy[safe]).all()
    else:
        qs = np.stack([oc.q_values(p, x.reshape(-1, 16)).reshape(q["T"], q["n"], 3) for p in dev])   # [K][T][n][3]
        srt = np.sort(qs, axis=-1)
        safe = (srt[..., 2] - srt[..., 1] > 2 * TOL_BF16).all(axis=0)
        votes = np.stack([(oc.first_argmax(qs) == j).sum(0) for j in range(3)], -1).astype(np.float32) / np.float32(K)
        assert (np.abs(prob - votes)[safe] == 0).all()
        safe &= ~explored
        assert (act[safe] == greedy[safe]).all()
    return safe.mean()


CASES = [dict(n=1, T=257, start=100, stride=0, key=11), dict(n=70, T=300, start=200, stride=37, key=12),
         dict(n=130, T=150, start=5000, stride=3, key=13)]


@pytest.mark.parametrize("rule,K,rows", [(0, 5, 64), (0, 3, 16), (1, 5, 16), (1, 1, 64)])
def test_parity_against_oracle(market, rule, K, rows):
    eps = 0.05
    srv, actors = _server(market, K=K, rule=rule, eps=eps, rows=rows, chunk=100)
    ids = [srv.submit(q["n"], q["T"], q["start"], q["stride"], q["key"], store_act=True, store_prob=True)
           for q in CASES]
    done = srv.run_all()
    assert sorted(done) == sorted(ids)
    for rid, q in zip(ids, CASES):
        res, act, prob = srv.result(rid)
        print(f"rule {rule} K {K} rows {rows} request n={q['n']} T={q['T']}", flush=True)
        frac = _check_request(market, actors, q, res, act.astype(np.int64), prob, rule, eps)
        assert frac > 0.3
    srv.close()


@pytest.mark.parametrize("eps,fee,rule,K", [(1.0, 2e-4, 0, 3), (0.0, 0.0, 1, 5)])
def test_degenerate_requests(market, eps, fee, rule, K):
    """Every action explored (eps = 1) or none (eps = 0, with no fee); a one-tick horizon; tiles
    filled exactly and by one environment more; a request whose last mark is the table's last tick."""
    n_ticks = len(market.mid)
    edge = dict(n=3, T=40, stride=5, key=33)
    edge["start"] = n_ticks - 1 - edge["T"] - edge["stride"] * (edge["n"] - 1)
    cases = [dict(n=64, T=1, start=0, stride=0, key=31), dict(n=65, T=130, start=64, stride=1, key=32), edge]
    srv, actors = _server(market, K=K, rule=rule, eps=eps, rows=64, chunk=64, fee=fee)
    ids = [srv.submit(q["n"], q["T"], q["start"], q["stride"], q["key"], store_act=True, store_prob=True)
           for q in cases]
    assert sorted(srv.run_all()) == sorted(ids)
    for rid, q in zip(ids, cases):
        res, act, prob = srv.result(rid)
        print(f"eps {eps} fee {fee} rule {rule} K {K} request n={q['n']} T={q['T']} start={q['start']}", flush=True)
        _check_request(market, actors, q, res, act.astype(np.int64), prob, rule, eps, fee=fee)
        # The rewards telescope: the final value is cash0 plus their sum, up to rounding.
        assert np.allclose(res["value"] - 1e5, res["sum_r"], rtol=0, atol=1e-6)
    srv.close()


def test_batch_invariance(market):
    """One request alone, then among others arriving at different chunk boundaries, then with a
    different chunk length: bit-identical results, actions and probabilities."""
    A = dict(n=100, T=500, start=300, stride=17, key=99)
    others = [dict(n=5, T=900, start=1000, stride=1, key=1), dict(n=300, T=200, start=50, stride=20, key=2),
              dict(n=64, T=333, start=7000, stride=4, key=3), dict(n=1, T=1000, start=9000, stride=0, key=4)]

    def run(chunk, mix):
        srv, _ = _server(market, chunk=chunk)
        rid = None
        if not mix:
            rid = srv.submit(A["n"], A["T"], A["start"], A["stride"], A["key"], store_act=True, store_prob=True)
            srv.run_all()
        else:
            for q in others[:2]:
                srv.submit(q["n"], q["T"], q["start"], q["stride"], q["key"])
            srv.step()
            srv.step()
            rid = srv.submit(A["n"], A["T"], A["start"], A["stride"], A["key"], store_act=True, store_prob=True)
            srv.step()
            for q in others[2:]:
                srv.submit(q["n"], q["T"], q["start"], q["stride"], q["key"])
            srv.run_all()
        out = srv.result(rid)
        srv.close()
        return out

    base = run(128, False)
    for chunk, mix in [(128, True), (77, True), (500, False)]:
        got = run(chunk, mix)
        assert got[0].tobytes() == base[0].tobytes(), (chunk, mix)
        assert (got[1] == base[1]).all() and got[2].tobytes() == base[2].tobytes(), (chunk, mix)


def test_admission_by_pool_bytes(market):
    """A pool that holds one 100-environment request at a time still serves three of them, in
    arrival order, with the same results as alone."""
    from paper_2501_10709_amd import binding as B
    pool = B.fm_serve_request_bytes(100)
    srv, _ = _server(market, chunk=64, pool_bytes=pool)
    qs = [dict(n=100, T=150 + 10 * i, start=100 + 50 * i, stride=9, key=20 + i) for i in range(3)]
    ids = [srv.submit(q["n"], q["T"], q["start"], q["stride"], q["key"]) for q in qs]
    active, queued = srv.step()
    assert (active, queued) == (1, 2)
    done = srv.run_all()
    assert done == ids
    got = [srv.result(i)[0] for i in ids]
    srv.close()
    for q, g in zip(qs, got):
        srv2, _ = _server(market, chunk=64)
        rid = srv2.submit(q["n"], q["T"], q["start"], q["stride"], q["key"])
        srv2.run_all()
        assert srv2.result(rid)[0].tobytes() == g.tobytes()
        srv2.close()


def test_request_validation(market):
    from paper_2501_10709_amd import binding as B
    srv, _ = _server(market, pool_bytes=B.fm_serve_request_bytes(50))
    with pytest.raises(B.FmError):
        srv.submit(10, 19_990, 5, 1, 0)       # past the end of the tick table
    with pytest.raises(B.FmError):
        srv.submit(60, 10, 100, 1, 0)         # larger than the pool
    srv.close()


def test_poisson_serving_loop_completes_every_request(market):
    """The continuous-batching loop (submissions at Poisson arrival times, steps, completions):
    every request completes once, with latencies at least its own compute time and results equal
    to running it alone."""
    from paper_2501_10709_amd.serve import serve_poisson
    from workload.crypto import poisson_requests
    reqs = poisson_requests(8, 12, 2000.0, market.n_ticks, n_range=(1, 200), horizon_range=(50, 400))
    srv, _ = _server(market, chunk=64)
    lat, makespan, steps = serve_poisson(srv, reqs)
    srv.close()
    assert lat.shape == (12,) and (lat > 0).all() and makespan > 0
    assert steps == sum(q.n_envs * q.horizon for q in reqs)
    q = reqs[3]
    srv1, _ = _server(market, chunk=64)
    a = srv1.submit(q.n_envs, q.horizon, q.start_tick, q.stride, q.key)
    srv1.run_all()
    alone = srv1.result(a)[0]
    srv1.close()
    srv2, _ = _server(market, chunk=64)
    ids = [srv2.submit(r.n_envs, r.horizon, r.start_tick, r.stride, r.key) for r in reqs[:6]]
    srv2.run_all()
    assert srv2.result(ids[3])[0].tobytes() == alone.tobytes()
    srv2.close()
