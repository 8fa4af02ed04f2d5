"""Rollout throughput on one MI355X: env-steps/s of the trading-environment rollout.

One step of the benchmark is one whole rollout of the hot path over one batch: reset, then
T = 252 days of (ensemble MLP forward -> noise -> orders -> sells -> buys -> next day's prices
and indicators -> reward -> next state), storing the state, action and reward trajectories as
[T][N][.] device tensors.  The workload is N = 2048 environments, D = 30 stocks, I = 5
indicators, K = 3 actors 211 -> 256 -> 256 -> 30.

Reported:
  value        env-steps/s (N*T / median rollout time) of the fused bfloat16 path
  fp32_plain   the same for the plain float32 path (per-step MLP and environment launches)
  latency_ms   p50 / p99 rollout latency of both paths
  roofline     the fused kernel against the bfloat16 MFMA peak: algorithmic flops per launch
               (763,392 per env-step x envs x steps of the launch) over the average launch time,
               timed with HIP events on the stream the kernels run on (the rollout launches one
               fused kernel per chunk of up to 64 steps)
  env_roofline the driven-mode environment kernel against HBM peak (1,092 B per env-step), at the
               headline size and at a size that fills the GPU (N = 65536, T = 64)
  cpu_baseline the CPU oracle (float64 numpy) on a bounded sample of the same workload
`traffic` comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs summarised in profiles/traffic.json,
scaled by the counters' reading for a copy kernel of known size; it is null when the kernel
sources have changed since those runs (a hash of the sources is stored with the numbers).
Inputs are generated on the host and uploaded before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s at N=2048,D=30 (BF16 fused vs FP32 plain); p50/p99 rollout latency"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0


def mlp_flops_per_env_step(S, H, A, K):
    """2 * (S*H + H*H + H*A) per actor: the algorithmic multiply-adds of the three layers."""
    return 2 * K * (S * H + H * H + H * A)


def env_bytes_per_env_step(D, S):
    """Driven rollout with state, reward and quantity trajectories: action read (4D), state write
    (4S), reward write (8), executed-quantity write (4D).  The per-env state stays on chip."""
    return 4 * D + 4 * S + 8 + 4 * D


CHUNK = 64  # steps per fused-kernel launch (the library's chunk)


# Sources the stock-environment and fused-rollout kernels (and their launch choices) are built from.
PROFILED_SOURCES = ("api.hip", "crypto_serve.hip", "device_common.h", "ensemble_kernels.hip", "env_kernels.hip",
                    "env_lane.hip",
                    "fused_resident.hip",
                    "fused.h", "fused_rollout.hip", "launch.h", "mlp_device.h", "row_chain.h", "status.h")


def source_hash():
    """Hash of the profiled HIP sources: counter readings are only valid for the code they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2501_10709_amd", "csrc")
    for name in PROFILED_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key, per_launch_units):
    """HBM bytes per launch from the committed counter summary, or None if stale or absent."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash() or kernel_key not in t.get("kernels", {}):
        return None
    k = t["kernels"][kernel_key]
    return k["bytes_per_unit"] * per_launch_units


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def time_rollouts(env, n_steps, reps, warmup, stream, **kw):
    """Times reps rollouts (reset + rollout).  Returns (per-rollout ms list, rollout-call ms list)."""
    import torch
    out = None
    for _ in range(warmup):
        env.reset(return_obs=False)
        out = env.rollout(n_steps, out=out, **kw)
    torch.cuda.synchronize()
    totals, kernels = [], []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    t0 = time.perf_counter()
    for i in range(reps):
        a, b, c = ev[i]
        a.record(stream)
        env.reset(return_obs=False)
        b.record(stream)
        out = env.rollout(n_steps, out=out, **kw)
        c.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for a, b, c in ev:
        totals.append(a.elapsed_time(c))
        kernels.append(b.elapsed_time(c))
    return totals, kernels, wall, out


def time_launches(env, n_steps, reps, stream, **kw):
    """Per-launch durations of a rollout issued chunk by chunk (one fused launch per call).
    Returns a list of (steps, ms) over reps rollouts."""
    import torch
    out, res = None, []
    for _ in range(reps):
        env.reset(return_obs=False)
        evs = []
        for c0 in range(0, n_steps, CHUNK):
            n = min(CHUNK, n_steps - c0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out = env.rollout(n, out=None, **kw)
            b.record(stream)
            evs.append((n, a, b))
        torch.cuda.synchronize()
        res += [(n, a.elapsed_time(b)) for n, a, b in evs]
    return res


def bench_precision(dev, w, args):
    """The precision form: N=8192, D=30, T=252, bfloat16 fused path (streamed schedule, the
    default at this size; the resident schedule timed beside it), states, actions and rewards
    stored.  The action and episode-return errors against the oracle are measured by the GPU
    test suite, not here."""
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    from workload import make_actor_weights, make_market, pack_actor_weights
    cfg, acfg = w.env, w.actors
    N, D, T, S, H, K = cfg.n_envs, cfg.n_stocks, cfg.n_days, cfg.state_dim, acfg.hidden, acfg.n_actors
    stream = torch.cuda.current_stream()
    m = make_market(w.market_seed, D, T)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    ens = Ensemble(pack_actor_weights(make_actor_weights(acfg)), K, S, H, D, dtype="bf16", max_batch=N, device=dev)
    kw = dict(ens=ens, sigma=w.sigma, noise_key=w.noise_key, path="fused", store=("obs", "act", "rew"))
    reps = max(5, args.steps // 3)
    out = {"workload": w.name, "dtype": "bf16",
           "schedule": "streamed (the default past one resident workgroup per compute unit)"}
    for name, schedule in (("streamed", 1), ("resident", 3)):
        env.set_fused_tuning(schedule=schedule)
        tot, _, _, _ = time_rollouts(env, T, reps, 2, stream, **kw)
        out[name] = {"value": N * T / (float(np.median(tot)) / 1e3), "unit": "env-steps/s",
                     "ms_per_rollout": float(np.median(tot)), "p50_ms": _pct(tot, 50), "p99_ms": _pct(tot, 99)}
    env.set_fused_tuning(schedule=0)
    launches = time_launches(env, T, 3, stream, **kw)
    flop = mlp_flops_per_env_step(S, H, D, K)
    steps = sum(n for n, _ in launches)
    ms = sum(t for _, t in launches)
    tf = flop * N * steps / (ms / 1e3) / 1e12
    out["value"] = out["streamed"]["value"]
    out["unit"] = "env-steps/s"
    out["roofline"] = {"bound": "mfma", "achieved": tf, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                       "frac": tf / PEAK_BF16_TFLOPS, "kernel": "fused_streamed_kernel",
                       "launch_ms": ms / len(launches), "steps_per_launch": steps / len(launches),
                       "launch_includes": "the chunk's market_table_kernel and noise_chunk_kernel",
                       "traffic": traffic_for("fused_streamed_kernel@8192", N * steps / len(launches))}
    del env, ens
    torch.cuda.empty_cache()
    return out


def bench_batched(dev, n_groups=64, reps=3):
    """The uneven batched form: 64 groups (D in {5,10,30,50,100}, N log-uniform 32..4096, T
    20..1000, per-group volatility), K=3 bfloat16 actors (7D+1)->256->256->D each, rewards stored;
    autotuned, chunk launches replayed from a hipGraph.  env-steps/s = sum N*T / median run time."""
    import torch
    from paper_2501_10709_amd.vecenv import Batch, Ensemble, VecEnv
    from workload import make_actor_weights, make_market, pack_actor_weights
    from workload.uneven import uneven_groups
    gs = uneven_groups(seed=4, n_groups=n_groups)
    made = []
    for g in gs:
        m = make_market(g.market_seed, g.env.n_stocks, g.env.n_days, vol=g.vol)
        env = VecEnv(g.env, m.close, m.ind, device=dev)
        ens = Ensemble(pack_actor_weights(make_actor_weights(g.actors)), 3, g.actors.in_dim, g.actors.hidden,
                       g.env.n_stocks, dtype="bf16", max_batch=g.env.n_envs, device=dev)
        made.append((g, env, ens))
        env.reset(return_obs=False)
    spec = [dict(env=env, ens=ens, n_steps=g.env.n_days, sigma=0.1, noise_key=7, env_offset=i * 4096, store=("rew",))
            for i, (g, env, ens) in enumerate(made)]
    batch = Batch(spec)
    rows, blocks = batch.tune()
    steps = sum(g.env.n_envs * g.env.n_days for g in gs)
    ts = []
    for _ in range(reps + 1):
        for _, env, _ in made:
            env.reset(return_obs=False)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        batch.run(use_graph=True)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts[1:]))
    batch.close()
    flops = sum(g.env.n_envs * g.env.n_days * mlp_flops_per_env_step(g.actors.in_dim, g.actors.hidden,
                                                                     g.env.n_stocks, 3) for g in gs)
    tf = flops / (ms / 1e3) / 1e12
    return {"workload": f"{n_groups} uneven groups, {steps} env-steps", "value": steps / (ms / 1e3),
            "unit": "env-steps/s", "ms": ms, "tile_rows": rows, "blocks": blocks, "graph": True,
            "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / PEAK_BF16_TFLOPS, "kernel": "fused_batched_kernel", "traffic": None,
                         "flop": flops, "flop_per_env_step": "2K(SH + H^2 + HA) of each group's shape"},
            "schedule": "generic (runtime shapes)"}


CRYPTO_FLOP_PER_ENV_STEP = 2 * 5 * (16 * 128 + 128 * 128 + 128 * 3)   # K=5 agents 16-128-128-3: 188,160


def crypto_server(dev, tick_seed=11, n_ticks=1_000_000, chunk=256, rows=64):
    from paper_2501_10709_amd.serve import CryptoServer
    from workload import pack_actor_weights
    from workload.crypto import crypto_actors, make_crypto_agents, make_ticks
    m = make_ticks(seed=tick_seed, n_ticks=n_ticks)
    W = pack_actor_weights(make_crypto_agents(crypto_actors()))
    return m, CryptoServer(m.mid, m.feat, W, 5, eps=0.005, fee=2e-4, tile_rows=rows, chunk_ticks=chunk,
                           device=dev)


def serving_capacity(srv, n_req=64, n_envs=4096, horizon=1024):
    """Saturated chunk launches: n_req requests of n_envs environments x horizon ticks admitted at
    once; every launch is timed with HIP events on the stream it runs on."""
    import torch
    stream = torch.cuda.current_stream()
    for i in range(n_req):
        srv.submit(n_envs, horizon, 1000 + 97 * i, 200, i)
    times, done = [], []
    while True:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        active, queued = srv.step()
        b.record(stream)
        times.append((a, b))
        done += srv.poll()
        if active == 0 and queued == 0:
            done += srv.poll(wait=True)
            break
    torch.cuda.synchronize()
    for rid in done:
        srv.requests.pop(rid, None)
    ms = [x.elapsed_time(y) for x, y in times]
    steps = n_req * n_envs * horizon
    tf = CRYPTO_FLOP_PER_ENV_STEP * steps / (sum(ms) / 1e3) / 1e12
    return {"workload": f"{n_req} requests x {n_envs} envs x {horizon} ticks admitted together",
            "env_steps_per_s": steps / (sum(ms) / 1e3), "launches": len(ms), "launch_ms": float(np.mean(ms)),
            "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / PEAK_BF16_TFLOPS,
                         "traffic": traffic_for("crypto_chunk_kernel<4,5>", steps / len(ms)),
                         "kernel": "crypto_chunk_kernel<4,5>",
                         "flop_per_env_step": CRYPTO_FLOP_PER_ENV_STEP}}


def bench_serving(dev, rate=200.0, n_requests=400):
    """Continuous-batching serving of the crypto task (Poisson arrivals, FIFO admission by pool
    bytes); p50/p99 request latency and throughput, and the saturated capacity."""
    from paper_2501_10709_amd.serve import serve_poisson
    from workload.crypto import poisson_requests
    m, srv = crypto_server(dev)
    cap = serving_capacity(srv)
    reqs = poisson_requests(5, n_requests, rate, m.n_ticks)
    offered = sum(q.n_envs * q.horizon for q in reqs)
    lat, makespan, steps = serve_poisson(srv, reqs)
    sweep = []
    for r in (100.0, 300.0):
        rq = poisson_requests(6, n_requests // 2, r, m.n_ticks)
        la, mk, st = serve_poisson(srv, rq)
        sweep.append({"rate_per_s": r, "requests": len(rq), "p50_ms": float(np.percentile(la, 50) * 1e3),
                      "p99_ms": float(np.percentile(la, 99) * 1e3), "throughput": st / mk,
                      "offered": sum(q.n_envs * q.horizon for q in rq) / rq[-1].arrival_s})
    srv.close()
    return {"workload": f"crypto serving: {m.n_ticks} ticks, K=5 bf16 agents 16-128-128-3 (averaged softmax), "
                        f"eps 0.005, Poisson {rate:g} req/s, {n_requests} requests, N log-uniform 1-4096, "
                        "horizon log-uniform 1k-100k ticks, 64-env tiles, 256-tick chunks",
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "throughput": steps / makespan, "unit": "env-steps/s", "offered": offered / reqs[-1].arrival_s,
            "makespan_s": makespan, "capacity": cap, "load_sweep": sweep}


def bench_learner(dev, w, reps=5):
    """The learner consuming a paper-scale rollout: the gradient of eqs. (4)-(5) for agent 0 from
    the stored [T][N] states and rewards (float32 master weights), per call."""
    import torch
    from paper_2501_10709_amd import binding as B
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    from workload import make_actor_weights, make_market, pack_actor_weights
    cfg, acfg = w.env, w.actors
    N, D, T, S, H, K = cfg.n_envs, cfg.n_stocks, cfg.n_days, cfg.state_dim, acfg.hidden, acfg.n_actors
    m = make_market(w.market_seed, D, T)
    packed = pack_actor_weights(make_actor_weights(acfg))
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    ens = Ensemble(packed, K, S, H, D, dtype="bf16", max_batch=N, device=dev)
    s0 = env.reset()
    out = env.rollout(T, ens=ens, sigma=w.sigma, noise_key=w.noise_key, path="fused", store=("obs", "rew"))
    states = torch.cat([s0[None], out["obs"][:-1]], 0).contiguous()
    rew = out["rew"].contiguous()
    del out
    wts = torch.as_tensor(packed).to(dev)
    per = S * H + H + H * H + H + H * D + D
    grad = torch.empty(per, dtype=torch.float32, device=dev)
    ws = torch.empty(B.fm_pg_workspace_bytes(K, S, H, D, N, T), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ts = []
    for i in range(reps + 2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        B.fm_policy_gradient(K, S, H, D, wts, 0, states, rew, N, T, w.sigma, w.noise_key, 0, 0.1, grad, ws)
        b.record(stream)
        torch.cuda.synchronize()
        if i >= 2:
            ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    rows = N * T
    flop = rows * (2 * K * (S * H + H * H + H * D) + 2 * (S * H + H * H + H * D) + 2 * (D * H + H * H))
    tf = flop / (ms / 1e3) / 1e12
    del ws, states, rew
    torch.cuda.empty_cache()
    return {"workload": f"policy gradient (eqs. 4-5, lambda 0.1) for one of {K} actors {S}-{H}-{H}-{D} from a "
                        f"{N} x {T} rollout", "ms": ms, "samples_per_s": rows / (ms / 1e3),
            "roofline": {"bound": "fp32", "achieved": tf, "peak": 157.3, "unit": "TFLOP/s", "frac": tf / 157.3,
                         "kernel": "gemm_kernel (float32 MFMA 16x16x4 tiles)", "flop_per_sample": flop / rows}}


def cpu_baseline(w, budget_s=10.0, max_reps=4):
    """The oracle (float64 numpy) on the same workload, timed on the host: whole closed-loop
    rollouts of all the workload's environments until about budget_s seconds of CPU work."""
    from oracle.rollout import rollout_closed_loop
    from workload import make_actor_weights, make_market
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    cfg = w.env
    m = make_market(w.market_seed, cfg.n_stocks, cfg.n_days)
    actors = make_actor_weights(w.actors)
    T = cfg.n_days
    reps, dt = 0, 0.0
    while reps < 1 or (dt < budget_s and reps < max_reps):
        t0 = time.perf_counter()
        rollout_closed_loop(cfg, m.close, m.ind, actors, T, w.sigma, w.noise_key)
        dt += time.perf_counter() - t0
        reps += 1
    return {"value": reps * cfg.n_envs * T / dt, "unit": "env-steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} closed-loop oracle rollout(s) of all {cfg.n_envs} envs x {T} days, "
                      f"float64 numpy, {dt:.1f} s", "host_cpus": os.cpu_count()}


def _oracle_shard(job):
    """One process's share of the sharded CPU baseline: a closed-loop oracle rollout of n envs with
    one BLAS thread.  Returns the seconds it took."""
    name, n = job
    from threadpoolctl import threadpool_limits
    from oracle.rollout import rollout_closed_loop
    from workload import WORKLOADS, make_actor_weights, make_market
    w = WORKLOADS[name]
    cfg = w.env
    m = make_market(w.market_seed, cfg.n_stocks, cfg.n_days)
    actors = make_actor_weights(w.actors)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        rollout_closed_loop(cfg, m.close, m.ind, actors, cfg.n_days, w.sigma, w.noise_key, n_envs=n)
        return time.perf_counter() - t0


def _noop(_):
    return 0


def cpu_baseline_sharded(key, procs=None):
    """The oracle with the environments split across processes (they are independent), one BLAS
    thread each.  Run before the GPU is touched: the pool's processes are started fresh."""
    import concurrent.futures
    import multiprocessing
    from workload import WORKLOADS
    w = WORKLOADS[key]
    procs = procs or os.cpu_count() or 1
    N, T = w.env.n_envs, w.env.n_days
    shares = [N // procs + (1 if i < N % procs else 0) for i in range(procs)]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(procs, mp_context=ctx) as ex:
        list(ex.map(_noop, range(procs)))              # start every worker first
        t0 = time.perf_counter()
        per = list(ex.map(_oracle_shard, [(key, n) for n in shares if n > 0]))
        dt = time.perf_counter() - t0
    return {"value": N * T / dt, "unit": "env-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"one closed-loop oracle rollout of {N} envs x {T} days split over {procs} processes "
                      f"(one BLAS thread each), {dt:.1f} s wall, slowest share {max(per):.1f} s"}


def hbm_copy_gbs(dev, nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth on this GPU: a 1 GiB device-to-device copy (read + write bytes)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (float(np.median(ts)) / 1e3) / 1e9


def profile_kernel(args):
    """One kernel family in isolation, for rocprofv3 (kernel trace or counters)."""
    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    from workload import WORKLOADS, make_actions, make_actor_weights, make_market, pack_actor_weights
    dev = torch.device("cuda:0")
    if args.kernel == "copy":
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"kernel": "copy", "bytes_read": nbytes, "bytes_written": nbytes}), flush=True)
        return
    if args.kernel == "batched":
        print(json.dumps(bench_batched(dev, reps=max(1, args.steps))), flush=True)
        return
    if args.kernel == "learner":
        print(json.dumps(bench_learner(dev, WORKLOADS[args.workload], reps=max(1, args.steps))), flush=True)
        return
    if args.kernel == "serve":
        _, srv = crypto_server(dev)
        print(json.dumps(serving_capacity(srv, n_req=max(1, args.steps) * 16)), flush=True)
        srv.close()
        return
    w = WORKLOADS[args.workload]
    cfg, acfg = w.env, w.actors
    N, D, T, S, H, K = cfg.n_envs, cfg.n_stocks, cfg.n_days, cfg.state_dim, acfg.hidden, acfg.n_actors
    m = make_market(w.market_seed, D, T)
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    kw = {}
    if args.kernel == "driven":
        kw = dict(actions=torch.from_numpy(make_actions(5, T, N, D)).to(dev), store=("obs", "rew", "qty"))
    else:
        dtype = "bf16" if args.kernel == "fused" else "f32"
        ens = Ensemble(pack_actor_weights(make_actor_weights(acfg)), K, S, H, D, dtype=dtype, max_batch=N,
                       device=dev)
        kw = dict(ens=ens, sigma=w.sigma, noise_key=w.noise_key, path="fused" if args.kernel == "fused" else "plain",
                  store=("obs", "act", "rew"))
    tot, ker, _, _ = time_rollouts(env, T, max(1, args.steps), 1, torch.cuda.current_stream(), **kw)
    print(json.dumps({"kernel": args.kernel, "workload": w.name, "rollout_ms": tot, "kernel_ms": ker,
                      "flop_per_env_step": mlp_flops_per_env_step(S, H, D, K),
                      "bytes_per_env_step": env_bytes_per_env_step(D, S), "env_steps": N * T}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper", choices=["paper", "precision", "envlarge"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-steps", type=int, default=None, help="timed rollouts of the plain float32 path")
    ap.add_argument("--kernel", choices=["fused", "driven", "plain", "copy", "batched", "serve", "learner"], default=None,
                    help="profiling mode: one warm-up and --steps launches of one kernel, nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the rollout shards by environment "
                                   "across GPUs with no communication, so N GPUs give N times one GPU's "
                                   "throughput and are not launched here"}))
        sys.exit(2)

    import torch
    from paper_2501_10709_amd.vecenv import Ensemble, VecEnv
    from workload import WORKLOADS, make_actor_weights, make_market, pack_actor_weights

    if args.kernel is not None:
        profile_kernel(args)
        return
    w = WORKLOADS[args.workload]
    sharded = None
    if not args.no_cpu_baseline:
        sharded = cpu_baseline_sharded(args.workload)
    cfg, acfg = w.env, w.actors
    N, D, T, S, H, K = cfg.n_envs, cfg.n_stocks, cfg.n_days, cfg.state_dim, acfg.hidden, acfg.n_actors
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = make_market(w.market_seed, D, T)
    packed = pack_actor_weights(make_actor_weights(acfg))

    # The driven environment kernel on a problem that fills the GPU (HBM-write bound), timed first,
    # before the compute-bound legs have run.
    from workload import make_actions
    wl = WORKLOADS["envlarge"]
    NL, TL = wl.env.n_envs, wl.env.n_days
    ml = make_market(wl.market_seed, D, TL)
    env_l = VecEnv(wl.env, ml.close, ml.ind, device=dev)
    acts_l = torch.rand((TL, NL, D), device=dev, dtype=torch.float32) * 2 - 1
    l_tot, l_ker, _, out_l = time_rollouts(env_l, TL, max(3, args.steps // 5), 1, stream, actions=acts_l,
                                           store=("obs", "rew", "qty"))
    del out_l, acts_l, env_l
    torch.cuda.empty_cache()
    env = VecEnv(cfg, m.close, m.ind, device=dev)
    store = ("obs", "act", "rew")
    ens_bf16 = Ensemble(packed, K, S, H, D, dtype="bf16", max_batch=N, device=dev)
    bf_tot, bf_ker, bf_wall, _ = time_rollouts(env, T, args.steps, args.warmup, stream, ens=ens_bf16,
                                               sigma=w.sigma, noise_key=w.noise_key, path="fused", store=store)
    launches = time_launches(env, T, max(3, args.steps // 5), stream, ens=ens_bf16, sigma=w.sigma,
                             noise_key=w.noise_key, path="fused", store=store)
    precision = bench_precision(dev, WORKLOADS["precision"], args)
    ens_f32 = Ensemble(packed, K, S, H, D, dtype="f32", max_batch=N, device=dev)
    f32_reps = args.fp32_steps if args.fp32_steps is not None else max(5, args.steps // 3)
    f_tot, f_ker, f_wall, _ = time_rollouts(env, T, f32_reps, max(1, args.warmup // 2), stream, ens=ens_f32,
                                            sigma=w.sigma, noise_key=w.noise_key, path="plain", store=store)

    # Driven-mode environment kernel (actions from HBM; states, rewards and quantities stored).
    acts = torch.from_numpy(make_actions(5, T, N, D)).to(dev)
    d_tot, d_ker, _, _ = time_rollouts(env, T, args.steps, args.warmup, stream, actions=acts,
                                       store=("obs", "rew", "qty"))
    del acts

    env_steps = N * T
    bf_ms = float(np.median(bf_tot))
    f_ms = float(np.median(f_tot))
    flop = mlp_flops_per_env_step(S, H, D, K) * env_steps
    ker_s = float(np.mean(bf_ker)) / 1e3
    flop_env_step = mlp_flops_per_env_step(S, H, D, K)
    launch_steps = sum(n for n, _ in launches)
    launch_ms = sum(ms for _, ms in launches)
    achieved_tf = flop_env_step * N * launch_steps / (launch_ms / 1e3) / 1e12
    mean_launch_ms = launch_ms / len(launches)
    steps_per_launch = launch_steps / len(launches)
    env_b = env_bytes_per_env_step(D, S) * env_steps
    d_s = float(np.median(d_ker)) / 1e3
    achieved_gbs = env_b / d_s / 1e9
    l_s = float(np.median(l_ker)) / 1e3
    large_gbs = env_bytes_per_env_step(D, S) * NL * TL / l_s / 1e9
    rec = {
        "metric": METRIC,
        "value": env_steps / (bf_ms / 1e3),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bf_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "n_envs": N, "n_stocks": D, "n_ind": cfg.n_ind, "n_days": T,
                   "actors": f"{K}x {S}-{H}-{H}-{D} tanh", "path": "fused bf16 MFMA, fp64 cash, int32 holdings",
                   "stored": list(store), "sigma": w.sigma},
        "latency_ms": {"bf16_fused_p50": _pct(bf_tot, 50), "bf16_fused_p99": _pct(bf_tot, 99),
                       "fp32_plain_p50": _pct(f_tot, 50), "fp32_plain_p99": _pct(f_tot, 99)},
        "fp32_plain": {"value": env_steps / (f_ms / 1e3), "unit": "env-steps/s", "ms_per_step": f_ms,
                       "steps": f32_reps, "dtype": "f32"},
        "bf16_over_fp32": f_ms / bf_ms,
        "roofline": {"bound": "mfma", "achieved": achieved_tf, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_BF16_TFLOPS,
                     "traffic": traffic_for("fused_resident_kernel", N * steps_per_launch),
                     "kernel": "fused_resident_kernel", "launch_ms": mean_launch_ms,
                     "launch_includes": "the chunk's market_table_kernel and noise_chunk_kernel",
                     "steps_per_launch": steps_per_launch, "flop_per_env_step": flop_env_step},
        "env_roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": achieved_gbs / PEAK_HBM_GBS,
                         "traffic": traffic_for("env_row_kernel<0>@2048", N * T),
                         "kernel": "env_row_kernel<0> (driven; the size-based choice at this N)",
                         "kernel_ms": d_s * 1e3, "us_per_step": d_s * 1e6 / T,
                         "bytes_per_env_step": env_bytes_per_env_step(D, S), "env_steps_per_s": env_steps / d_s,
                         "large": {"workload": wl.name, "achieved": large_gbs, "frac": large_gbs / PEAK_HBM_GBS,
                                   "kernel": "env_lane_kernel<0,32> (one lane per environment)",
                                   "kernel_ms": l_s * 1e3, "env_steps_per_s": NL * TL / l_s,
                                   "traffic": traffic_for("env_lane_kernel@65536", NL * TL)}},
    }
    rec["precision"] = precision
    rec["batched_uneven"] = bench_batched(dev)
    rec["serving"] = bench_serving(dev)
    rec["learner"] = bench_learner(dev, w)
    copy = hbm_copy_gbs(dev)
    rec["env_roofline"]["hbm_copy_GBs"] = copy
    rec["env_roofline"]["frac_of_copy"] = achieved_gbs / copy
    rec["env_roofline"]["large"]["frac_of_copy"] = large_gbs / copy
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
        rec["cpu_baseline_sharded"] = sharded
        c1 = cpu_baseline(WORKLOADS["tiny"], budget_s=3.0, max_reps=1000)
        c1["workload"] = WORKLOADS["tiny"].name
        rec["cpu_baseline_tiny"] = c1
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
