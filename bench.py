"""Throughput of the batched value-iteration path on one MI355X.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload 50x100]

Workload (seeded, synthetic; stands in for the paper's smart-warehouse models,
which are not available): 50 agents on 32x32..128x128 grids with 20 %
obstacles x 100 reach/avoid tasks of 3-12 DFA locations -> 5,000 agent-task
product MDPs, K = 64 weight columns per pass, eps 1e-6, FP32 backups with FP64
residual, polish, evaluation and reported values.

A step is one lockstep pass of Alg. 1 for 64 queries: the learned proposer's
first weights when present (plain: Dirichlet first weights), the batched
value iteration of all 5,000 models for the 64 columns to convergence (Alg. 3
and the stop test), the assignment (Alg. 2), FP64 polish, policy extraction
and per-objective evaluation of the assigned models (Alg. 4), and both
projections of Alg. 1 for every query.  `value` is state-action backups per
second over the timed steps (inputs resident on the device), which replay
captured graphs of sweep chunks; the kernel figures come from one more pass of
the same kind with HIP events around the sweep launches (eager launches).

Extra objects on the JSON line:
  roofline      the Bellman sweep kernel: algorithmic bytes (CSR of active
                models + one FP32 read and one write per active state-column)
                over its summed HIP-event durations, against 8 TB/s HBM; the
                last sweeps of a solve (under 20 % of the tiles active) run the
                LDS-staged kernel, reported apart as `tail_kernel`;
                `traffic` = HBM bytes per launch from the committed rocprofv3
                counter summary (profiles/sweep_traffic_50x100.txt), null when
                the sweep sources changed since it was taken;
  cpu_baseline  the FP64 oracle's value iteration timed on a bounded sample of
                models of the same workload on the host, one process per
                core used (8 by default);
  ms_per_query  Alg. 1 queries (eps 0.01, at most --query-max-iter passes,
                each pass's solve started from the previous pass's values) on
                the timed workload: latency p50 / p99, passes, verdicts, how
                many met the stop test; plain first weight (1, 0, ..., 0)
                against the learned proposer trained on the device from the
                plain method's support steps on other weight vectors of the
                same workload (thresholds around the point r(w) of a weight
                vector w, target w);
  proposer      learned vs plain first weight on the 10 x 20 family: the
                proposer is trained on the device from the plain method's
                support steps on seeded variants (thresholds around the
                point r(w) of a weight vector w, target w; 200k tuples), then
                both loops answer unseen thresholds.
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

HBM_PEAK_GBS = 8000.0
METRIC = "state-action backups/s + ms per point-oriented Pareto query (learned vs plain)"


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


SHAPES = [(1, 1), (1, 2), (2, 1), (1, 4), (2, 2), (4, 1), (1, 8), (2, 4), (4, 2), (1, 16), (2, 8),
          (4, 4), (1, 32), (2, 16), (4, 8), (1, 64), (2, 32), (4, 16)]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_50x100.txt")


def kernel_name(variant: int, prec: str) -> str:
    """Device symbol of a sweep variant as rocprofv3 prints it, up to the
    block kernels' sparsity-pattern argument."""
    if variant < 0:
        return "morap::k::inst_vi_kernel"
    t = "float" if prec == "f32" else "double"
    if variant in (39, 40):
        return f"void morap::k::bellman_halo<{2 if variant == 39 else 4}"
    cpl, lps = SHAPES[(variant - 1) % 18]
    if variant > 36:
        return f"void morap::k::bellman_block_wave<{t}, {2 if variant == 37 else 8}, 256"
    if variant > 18 and (cpl, lps) == (1, 64):
        return f"void morap::k::bellman_block_wave<{t}, 4, 256"
    if variant > 18:
        return f"void morap::k::bellman_block<{t}, {cpl}, {lps}, 2, 256"
    v2 = "HIP_vector_type<float, 2u>" if prec == "f32" else "HIP_vector_type<double, 2u>"
    return f"void morap::k::bellman_sweep<{t}, {v2}, {cpl}, {lps}, {min(256, 64 * lps)}>"


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it has none or the sweep sources changed since."""
    from paper_2305_04397_amd.profile_summary import sources_hash
    if not os.path.exists(TRAFFIC_FILE):
        return None
    lines = open(TRAFFIC_FILE).read().splitlines()
    src = [l.split(":", 1)[1].strip() for l in lines if l.startswith("kernel_source_sha256:")]
    if not src or src[0] != sources_hash():
        return None
    # the kernel the solves ran (most dispatches), not an autotuner candidate
    # of the same name prefix
    best = None
    for l in lines:
        parts = l.split(",", 4)
        if len(parts) == 5 and parts[4].startswith(kernel) and parts[0].isdigit():
            if best is None or int(parts[0]) > best[0]:
                best = (int(parts[0]), float(parts[3]))
    return None if best is None else best[1]


def query_stats(res, wall_ms: float, eps: float, morap) -> dict:
    """Summary of one lockstep batch of queries: latency to each query's last
    pass (p50 / p99), passes, verdicts, how many met the loop's stop test."""
    its = np.array([q["iterations"] for q in res])
    lat = np.array([q["latency_ms"] for q in res])
    gaps = np.array([q["gap"] for q in res])
    v = [q["verdict"] for q in res]
    return {"queries": len(res), "wall_ms": round(wall_ms, 1), "ms_per_query": round(wall_ms / len(res), 2),
            "latency_p50_ms": round(float(np.percentile(lat, 50)), 1),
            "latency_p99_ms": round(float(np.percentile(lat, 99)), 1),
            "passes_mean": round(float(its.mean()), 2), "passes_p50": float(np.median(its)),
            "passes_max": int(its.max()), "stopped_within_eps": int((gaps <= eps).sum()),
            "gap_p50": round(float(np.median(gaps)), 4),
            "feasible": v.count(morap.FEASIBLE), "infeasible": v.count(morap.INFEASIBLE),
            "undecided": v.count(morap.UNDECIDED),
            "backups": int(sum(q["backups"] for q in res))}


_SINGLE_CORE = r'''
import json, os, sys, time
os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})
sys.path.insert(0, sys.argv[1])
import numpy as np
from workloads import make_workload, dirichlet_weights
from oracle import product, alg
out = {}
for cfg, name in ((1, "2x2"), (2, "10x20")):
    wl = make_workload(cfg)
    t0 = time.perf_counter()
    prods = product.build_all(wl)
    build = time.perf_counter() - t0
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(3), 4, nI + nJ)
    t0 = time.perf_counter()
    for k, w in enumerate(W):
        r = alg.support(prods, nI, nJ, w, 1e-6).r
        print(f"[bench] single-core oracle {name}: support step {k + 1}/{len(W)} done", file=sys.stderr, flush=True)
    per = (time.perf_counter() - t0) / len(W)
    t = r - 0.05 * np.abs(r)
    t0 = time.perf_counter()
    q = alg.query(prods, nI, nJ, t, 0.01, 1e-6)
    out[name] = {"product_build_s": round(build, 3), "support_s_per_weight_vector": round(per, 3),
                 "query_s": round(time.perf_counter() - t0, 3), "query_passes": int(q.iterations)}
    print(f"[bench] single-core oracle {name}: {out[name]}", file=sys.stderr, flush=True)
print(json.dumps(out))
'''


def oracle_single_core() -> dict:
    """The FP64 oracle on one host core (one thread: BLAS threads 1, the
    process pinned to one core), on the 2 x 2 and 10 x 20 workloads in full:
    product construction, one support step (Alg. 2) per Dirichlet weight
    vector, and one query (Alg. 1, eps 0.01) just below a support point."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _SINGLE_CORE, ROOT], stdout=subprocess.PIPE, text=True, env=env,
                       timeout=1200)
    if r.returncode != 0:
        raise RuntimeError(f"single-core oracle run failed with status {r.returncode} (its stderr is above)")
    return json.loads(r.stdout.strip().splitlines()[-1])


def stage_retirement_eval(ctx, rng, K: int, d: int, eps: float) -> dict:
    """Value iteration of K Dirichlet weight columns on the loaded products,
    plain (morap_solve, graphs) and with stage retirement (morap_solve_staged,
    eager launches), in FP64 and in FP32: wall time of the second of two runs
    each, sweeps, backups and algorithmic bytes, and the largest change of a
    value at an initial state."""
    from paper_2305_04397_amd import morap
    W = rng.dirichlet(np.ones(d), size=K)
    out = {"K": K, "eps_vi": eps}
    for prec in ("f64", "f32"):
        o = morap.Options(eps_vi=eps, precision=prec)
        res, c = {}, {}
        for name, fn in (("plain", ctx.solve), ("staged", ctx.solve_staged)):
            for _ in range(2):
                t0 = time.perf_counter()
                c[name], st = fn(W, o)
                ms = (time.perf_counter() - t0) * 1e3
            res[name] = {"ms": round(ms, 1), "sweeps": st["sweeps"], "backups": st["backups"],
                         "bytes": st["bytes"] + st["bytes_tail"], "variant": st["variant"]}
            log(f"stage retirement {prec}: {name} {ms:.0f} ms, {st['sweeps']} sweeps, {st['backups']:.4e} backups")
        res["backups_saved"] = round(1.0 - res["staged"]["backups"] / res["plain"]["backups"], 4)
        res["max_rel_change_c"] = float(np.abs(c["staged"] - c["plain"]).max() / max(1.0, np.abs(c["plain"]).max()))
        out[prec] = res
    return out


def query_eval(ctx, wl, front, rng, args, eps_vi: float) -> dict:
    """ms per point-oriented Pareto query on the timed workload, plain and
    learned first weight.  Thresholds: half below front points (achievable),
    half around them.  The learned proposer for this workload's d is trained
    on the device from the plain method's support steps on other weight
    vectors of the same workload (thresholds drawn around the point r(w) of
    a weight vector w, target w), then answers the same thresholds as the
    plain loop."""
    from paper_2305_04397_amd import morap, proposer_data as pdata
    nI, d = wl.n_agents, wl.n_agents + wl.n_tasks
    opts = morap.Options(eps_vi=eps_vi, precision=args.precision, eval_from_values=not args.eval_from_zero)
    loop_eps = 0.01
    T = pdata.thresholds(rng, front, args.queries, nI, inside_half=True)
    out = {"workload": wl.name, "eps": loop_eps, "max_iter": args.query_max_iter,
           "thresholds": "half below front points, half around them (U[-0.3, 0.3] per coordinate)",
           "warm_started_passes": True}
    tq = time.perf_counter()
    plain = ctx.query_batch(T, max_iter=args.query_max_iter, eps=loop_eps, opts=opts)
    out["plain"] = query_stats(plain, (time.perf_counter() - tq) * 1e3, loop_eps, morap)
    log(f"queries plain: {out['plain']}")
    out["learned"] = None
    if args.query_train > 0:
        t0 = time.perf_counter()
        phi = pdata.features(ctx, wl, opts)
        X, Wt = pdata.generate_from_support(ctx, wl, args.query_train, 2, phi, rng, opts)
        gen_s = time.perf_counter() - t0
        ctx.proposer_init(X.shape[1], d, seed=args.seed)
        ctx.proposer_set_input_norm(X.mean(0), X.std(0) + 1e-3)
        tt = time.perf_counter()
        losses = ctx.proposer_train(X, Wt, batch=64, epochs=200, lr=1e-3, seed=args.seed)
        train_s = time.perf_counter() - tt
        ctx.set_features(phi)
        tq = time.perf_counter()
        learned = ctx.query_batch(T, max_iter=args.query_max_iter, eps=loop_eps, opts=opts, use_proposer=True)
        out["learned"] = query_stats(learned, (time.perf_counter() - tq) * 1e3, loop_eps, morap)
        out["learned"].update({"train_tuples": int(len(X)), "data_s": round(gen_s, 1),
                               "train_s": round(train_s, 2), "loss_first": round(float(losses[0]), 4),
                               "loss_last": round(float(losses[-1]), 4),
                               "fallbacks": int(sum(q["fallback"] == 1 for q in learned))})
        decided = [(p, q) for p, q in zip(plain, learned)
                   if p["verdict"] != morap.UNDECIDED and q["verdict"] != morap.UNDECIDED]
        out["learned_vs_plain_verdicts"] = f"{sum(p['verdict'] == q['verdict'] for p, q in decided)}/{len(decided)}"
        log(f"queries learned: {out['learned']}")
    return out


_CPU_WL = None   # the workload, inherited by the forked baseline workers


def _cpu_worker(task):
    """One worker of the CPU baseline: FP64 oracle value iteration on models
    drawn at random (its own stream) until `budget_s` of VI time."""
    from threadpoolctl import threadpool_limits
    from oracle import product, vi
    threadpool_limits(1)                      # one core per process
    K, eps, budget_s, seed, worker = task
    wl = _CPU_WL
    rng = np.random.default_rng([seed, worker])
    nI, nJ = wl.n_agents, wl.n_tasks
    W = np.random.default_rng(seed).dirichlet(np.ones(nI + nJ), size=K)
    backups, elapsed, done = 0, 0.0, 0
    for m in rng.permutation(nI * nJ):
        i, j = divmod(int(m), nJ)
        if wl.agents[i].n_states > 2000:      # keep the sample bounded: agents of at most 2,000 cells
            continue
        p = product.build_product(wl.agents[i], wl.tasks[j], wl.letters[i][j])
        t0 = time.perf_counter()
        _, sweeps = vi.value_iteration(p, W[:, i], W[:, nI + j], eps)
        elapsed += time.perf_counter() - t0
        backups += int(sweeps.sum()) * p.n_rows
        done += 1
        if elapsed >= budget_s:
            break
    return backups, elapsed, done


def cpu_baseline(wl, K: int, eps: float, budget_s: float, seed: int, workers: int) -> dict:
    """The FP64 oracle's value iteration on a bounded sample of the workload's
    models, one process per host core used (forked before the GPU is
    touched).  value = sum over workers of backups / VI seconds."""
    import multiprocessing as mp
    global _CPU_WL
    _CPU_WL = wl
    tasks = [(K, eps, budget_s, seed, w) for w in range(workers)]
    if workers == 1:
        res = [_cpu_worker(tasks[0])]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_cpu_worker, tasks)
    rate = sum(b / e for b, e, _ in res if e > 0)
    done = sum(d for _, _, d in res)
    return {"value": rate, "unit": "backups/s", "cores": workers, "kind": "oracle",
            "per_core": rate / workers, "host_cpus": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0)),
            "sample": f"{done} models drawn at random from the workload (agents of at most 2,000 cells) by {workers} "
                      f"processes, K={K} Dirichlet weight columns, eps {eps:g}, FP64 Jacobi value iteration "
                      f"(numpy/scipy), about {budget_s:.0f} s of VI per process"}


def proposer_eval(args) -> dict:
    """Learned vs plain first weight on the 10 x 20 family (d = 30).

    The plain method's support steps on seeded 10 x 20 variants give
    (threshold, weight) tuples: thresholds drawn around the point r(w) that
    the support step returned for a Dirichlet weight vector w, with w as the
    target; the proposer is trained on them on the device, then both loops
    answer the same unseen thresholds of variant 0 (fresh draws, half of them
    achievable): wall time and Alg. 2 passes per query, and agreement of the
    answers."""
    from workloads import make_workload
    from paper_2305_04397_amd import morap, proposer_data as pdata
    rng = np.random.default_rng(args.seed + 1)
    opts = morap.Options(eps_vi=1e-6, precision="f32", eval_from_values=not args.eval_from_zero)
    ctx = morap.Context(0)
    X, Wt, phis, eval_T = [], [], {}, None
    t0 = time.perf_counter()
    per_variant = max(1, args.proposer_train // (2 * args.proposer_variants))
    for v in range(args.proposer_variants):
        wl = make_workload(2, variant=v)
        ctx.build_products(wl)
        phi = pdata.features(ctx, wl, opts)
        x, w = pdata.generate_from_support(ctx, wl, per_variant, 2, phi, rng, opts)
        X.append(x)
        Wt.append(w)
        if v == 0:
            phis[0] = phi
            front = pdata.front_points(ctx, wl, 256, rng, opts)
            eval_T = pdata.thresholds(rng, front, args.proposer_queries, wl.n_agents, inside_half=True)
        log(f"proposer data: variant {v}, {len(x)} tuples ({time.perf_counter() - t0:.0f} s)")
    X, Wt = np.vstack(X), np.vstack(Wt)
    d = Wt.shape[1]
    ctx.proposer_init(X.shape[1], d, seed=args.seed)
    ctx.proposer_set_input_norm(X.mean(0), X.std(0) + 1e-3)
    tt = time.perf_counter()
    losses = ctx.proposer_train(X, Wt, batch=256, epochs=80, lr=1e-3, seed=args.seed)
    train_s = time.perf_counter() - tt
    log(f"proposer trained on {len(X)} tuples in {train_s:.1f} s: loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    # evaluation on variant 0
    wl = make_workload(2, variant=0)
    ctx.build_products(wl)
    ctx.set_features(phis[0])
    ctx.query_batch(eval_T[:8], eps=0.01, opts=opts)                         # warm caches
    out = {"workload": wl.name, "eps": 0.01, "train_tuples": int(len(X)),
           "train_data": "support points r(w) of Dirichlet weight vectors w, two thresholds around each, target w",
           "train_variants": args.proposer_variants, "epochs": 80, "train_s": round(train_s, 2),
           "loss_first": round(float(losses[0]), 4), "loss_last": round(float(losses[-1]), 4)}
    res = {}
    # plain; the proposer's first weight vector; the proposer's weight vector
    # at every pass (input t_down after the first; a query keeps Alg. 1's
    # update once a proposal is invalid, repeats a weight vector or the
    # previous learned pass did not shrink the gap by 1 %)
    for name, use, passes in (("plain", False, 1), ("learned", True, 1), ("learned_every_pass", True, 64)):
        ts = time.perf_counter()
        r = ctx.query_batch(eval_T, eps=0.01, opts=opts, use_proposer=use, proposer_passes=passes)
        ms = (time.perf_counter() - ts) * 1e3
        its = np.array([q["iterations"] for q in r])
        res[name] = r
        out[name] = {"queries": len(r), "wall_ms": round(ms, 1), "ms_per_query": round(ms / len(r), 3),
                     "passes_mean": round(float(its.mean()), 3), "passes_max": int(its.max())}
        if use:
            out[name]["first_weight_fallbacks"] = int(sum(q["fallback"] == 1 for q in r))
            out[name]["later_weight_fallbacks"] = int(sum(q["fallback"] == 2 for q in r))
        log(f"proposer eval {name}: {ms / len(r):.2f} ms/query, passes mean {its.mean():.2f}")
    # verdicts are compared where both loops decided; a threshold within eps
    # of the front may end UNDECIDED in one loop and decided in the other
    decided = [(p, q) for p, q in zip(res["plain"], res["learned"])
               if p["verdict"] != morap.UNDECIDED and q["verdict"] != morap.UNDECIDED]
    agree = sum(p["verdict"] == q["verdict"] for p, q in decided)
    out["verdict_agreement"] = f"{agree}/{len(decided)}"
    out["undecided_in_either"] = len(eval_T) - len(decided)
    decided3 = [(p, q) for p, q in zip(res["plain"], res["learned_every_pass"])
                if p["verdict"] != morap.UNDECIDED and q["verdict"] != morap.UNDECIDED]
    out["verdict_agreement_every_pass"] = f"{sum(p['verdict'] == q['verdict'] for p, q in decided3)}/{len(decided3)}"
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="50x100", choices=["50x100", "10x20"])
    ap.add_argument("--queries", type=int, default=64, help="queries for the ms-per-query measurement (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="VI seconds per baseline process")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="baseline processes (at most the cores this process may run on)")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--schedule", type=int, default=0,
                    help="sweep-kernel variant of the timed passes (0 = the autotuner's choice)")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--no-graph", action="store_true",
                    help="timed steps enqueue every launch instead of replaying captured graphs (profiler runs)")
    ap.add_argument("--query-max-iter", type=int, default=48,
                    help="Alg. 2 passes allowed per query in the ms-per-query measurement")
    ap.add_argument("--query-train", type=int, default=2048,
                    help="support points (two thresholds each) training the learned proposer on the timed "
                         "workload (0 = skip)")
    ap.add_argument("--proposer-queries", type=int, default=1000,
                    help="unseen 10x20 queries for the learned-vs-plain comparison (0 = skip)")
    ap.add_argument("--proposer-train", type=int, default=200_000,
                    help="training tuples over the 10x20 variants (support points, two thresholds each)")
    ap.add_argument("--proposer-variants", type=int, default=4)
    ap.add_argument("--eval-from-zero", action="store_true",
                    help="start every policy evaluation (Alg. 4) from 0 instead of the solve's values")
    ap.add_argument("--stage-retirement", action="store_true",
                    help="also compare FP64 value iteration with and without stage retirement on the workload")
    ap.add_argument("--oracle-single-core", action="store_true",
                    help="also time the FP64 oracle on one core on the 2x2 and 10x20 workloads in full (~2 min)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X (multi-GPU sharding is "
              "described in DESIGN.md, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from workloads import make_workload
    from paper_2305_04397_amd import morap, proposer_data as pdata

    cfg = 3 if args.workload == "50x100" else 2
    K = 64 if cfg == 3 else 16
    eps = 1e-6
    t0 = time.time()
    wl = make_workload(cfg)
    nI, nJ = wl.n_agents, wl.n_tasks
    d = nI + nJ
    log(f"workload {wl.name}: generated in {time.time() - t0:.1f} s")
    # the CPU baseline first: its worker processes fork before the GPU is used
    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(args.cpu_workers, len(os.sched_getaffinity(0))))
        cpu = cpu_baseline(wl, K, eps, args.cpu_seconds, args.seed, workers)
        log(f"cpu baseline: {cpu['value']:.3e} backups/s on {workers} processes")
    if args.oracle_single_core:
        single = oracle_single_core()
        log(f"oracle on one core: {single}")
        if cpu is None:
            cpu = {"kind": "oracle"}
        cpu["single_core_full_workloads"] = single
    ctx = morap.Context(0)
    t0 = time.time()
    ctx.build_products(wl)
    tot = ctx.model_info(0)["total_states"]
    S = R = N = 0
    for m in range(nI * nJ):
        info = ctx.model_info(m)
        S, R, N = S + info["n_states"], R + info["n_rows"], N + info["nnz"]
    log(f"{nI * nJ} products built and uploaded in {time.time() - t0:.1f} s: S={S} R={R} N={N}")
    # the timed steps replay captured graphs of sweep chunks; one extra pass
    # with HIP events around the sweep launches (eager) gives the kernel figures
    # Alg. 4 starts from the solve's scalarised values (--eval-from-zero: from 0)
    efv = not args.eval_from_zero
    opts = morap.Options(eps_vi=eps, precision=args.precision, schedule=args.schedule, use_graph=not args.no_graph,
                         eval_from_values=efv)
    opts_timed = morap.Options(eps_vi=eps, precision=args.precision, time_kernels=True, schedule=args.schedule,
                               eval_from_values=efv)
    rng = np.random.default_rng(args.seed)

    # warm-up (includes the sweep-kernel autotuning) and front points
    fronts = []
    for w in range(args.warmup):
        Wd = rng.dirichlet(np.ones(d), size=K)
        r, _, _, st = ctx.support(Wd, opts)
        fronts.append(r)
        log(f"warmup {w + 1}/{args.warmup}: {st['ms_total']:.0f} ms, variant {st['variant']}, "
            f"{st['sweeps']} sweeps")
    if not fronts:
        r, _, _, _ = ctx.support(rng.dirichlet(np.ones(d), size=K), opts)
        fronts.append(r)
    front = np.vstack(fronts)

    # timed steps: one lockstep Alg. 1 pass of K queries each
    ctx.reset_stats()
    step_ms = []
    t_all = time.perf_counter()
    for s in range(args.steps):
        T = pdata.thresholds(rng, front, K, nI)
        W0 = rng.dirichlet(np.ones(d), size=K)
        ts = time.perf_counter()
        ctx.query_batch(T, W0=W0, max_iter=1, eps=0.01, opts=opts)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        log(f"step {s + 1}/{args.steps}: {step_ms[-1]:.0f} ms")
    wall = time.perf_counter() - t_all
    st_graph = ctx.stats()
    value = st_graph["backups"] / wall
    # one more pass of the same kind with HIP events on the library's stream
    # around every 4th sweep launch (a uniform sample; eager launches)
    ctx.reset_stats()
    T = pdata.thresholds(rng, front, K, nI)
    W0 = rng.dirichlet(np.ones(d), size=K)
    ts = time.perf_counter()
    ctx.query_batch(T, W0=W0, max_iter=1, eps=0.01, opts=opts_timed)
    timed_pass_ms = (time.perf_counter() - ts) * 1e3
    st = ctx.stats()
    log(f"kernel-timed pass (eager launches): {timed_pass_ms:.0f} ms")
    # dominant kernel: the FP32 batched sweep over all (model, column) pairs
    # until few tiles stay active: bytes per launch over its launches,
    # duration averaged over its timed ones
    main_sweeps = st["sweeps"] - st["sweeps_tail"]
    per_launch_bytes = st["bytes"] / max(1, main_sweeps)
    avg_s = st["ms_sweep_kernel"] / 1e3 / max(1, st["sweep_launches"])
    achieved = per_launch_bytes / avg_s / 1e9 if st["ms_sweep_kernel"] > 0 else 0.0
    kname = kernel_name(st["variant"], args.precision)
    tb = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if tb is None else round(tb, 0),
                "kernel": kname, "variant": st["variant"], "launches": main_sweeps,
                "launches_timed": st["sweep_launches"],
                "avg_launch_us": round(st["ms_sweep_kernel"] * 1e3 / max(1, st["sweep_launches"]), 2),
                "bytes_per_launch": round(per_launch_bytes, 0),
                "timing": "HIP events on every 4th sweep launch of one extra pass (eager launches); value and "
                          "ms_per_step come from the timed steps, which replay captured graphs"}
    if st["sweeps_tail"]:
        avg_t = st["ms_sweep_kernel_tail"] / 1e3 / max(1, st["sweep_launches_tail"])
        bt = st["bytes_tail"] / st["sweeps_tail"]
        roofline["tail_kernel"] = {
            "kernel": kernel_name(st["variant_tail"], args.precision), "variant": st["variant_tail"],
            "launches": st["sweeps_tail"], "launches_timed": st["sweep_launches_tail"],
            "avg_launch_us": round(avg_t * 1e6, 2), "bytes_per_launch": round(bt, 0),
            "achieved": round(bt / avg_t / 1e9, 1) if avg_t > 0 else None,
            "traffic": measured_traffic(kernel_name(st["variant_tail"], args.precision)),
            "note": "the last sweeps of each solve (under 20 % of the tiles active) run the LDS-staged kernel"}
    if st["sweep_launches_refine"]:
        avg_r = st["ms_sweep_kernel_refine"] / 1e3 / st["sweep_launches_refine"]
        ach_r = st["bytes_refine"] / max(1, st["polish_sweeps"]) / avg_r / 1e9
        roofline["fp64_assigned_resolve"] = {
            "achieved": round(ach_r, 1), "launches": st["polish_sweeps"],
            "launches_timed": st["sweep_launches_refine"], "avg_launch_us": round(avg_r * 1e6, 2),
            "kernel": kernel_name(st["variant_refine"], "f64")}
    log(f"timed: {value:.3e} backups/s, {float(np.mean(step_ms)):.0f} ms per step; sweep kernel {achieved:.0f} GB/s "
        f"({main_sweeps} launches, {st['sweep_launches']} timed, {st['ms_sweep_kernel']:.0f} ms; then "
        f"{st['sweeps_tail']} of the tail kernel, {st['ms_sweep_kernel_tail']:.0f} ms); FP64 re-solve "
        f"{st['ms_sweep_kernel_refine']:.0f} ms over {st['sweep_launches_refine']} timed launches; "
        f"VI {st['ms_vi']:.0f} ms, evaluation {st['ms_eval']:.0f} ms")

    # full queries on the timed workload: plain and learned first weight
    per_query = query_eval(ctx, wl, front, rng, args, eps) if args.queries > 0 else None
    staged = stage_retirement_eval(ctx, rng, K, d, eps) if args.stage_retirement else None

    ctx.close()
    learned = None
    if args.proposer_queries > 0:
        learned = proposer_eval(args)


    line = {"metric": METRIC, "value": value, "unit": "backups/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(float(np.mean(step_ms)), 2), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
            "data": "synthetic: seeded grid-world agents and reach/avoid task automata",
            "config": {"workload": f"{wl.name}: {nI * nJ} product MDPs, K={K} weight columns per pass",
                       "states": S, "rows": R, "nnz": N, "K": K, "eps_vi": eps, "seed": args.seed,
                       "eval_start": "from 0" if args.eval_from_zero else "from the solve's values",
                       "parallelism": "1 GPU"},
            "roofline": roofline, "cpu_baseline": cpu, "ms_per_query": per_query,
            "proposer": learned, "stage_retirement": staged,
            "stats": {k: st_graph[k] for k in ("backups", "sweeps", "sweeps_tail", "eval_sweeps", "polish_sweeps",
                                               "rank_rounds", "floor_stops", "ms_vi", "ms_eval", "variant",
                                               "variant_tail", "variant_refine", "bytes", "bytes_tail",
                                               "bytes_refine", "refine_pairs", "refine_columns")}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
