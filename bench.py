#!/usr/bin/env python3
"""Throughput of the local diffusion solvers on one MI355X.

Default workload (PPR on the n = 10^6 power-law graph): undirected Chung-Lu
graph, n = 1,000,000, 10,000,000 edges (nnz 2e7), degree exponent 2.5, RNG seed
42, int32 CSR, FP32 x / r.  One step = 64 seed nodes (uniform over the largest
component) x eps in {1e-4, 1e-5, 1e-6, 1e-7} x {LocalGD, LocalCH}, PPR
alpha = 0.1, each query solved on its own through the C ABI (the plain path),
outputs left in HBM.

Printed: one JSON line with solves/s (value), the algorithmic HBM GB/s of the
whole step, per-solve latency p50 / p99, the roofline of the dominant kernel
(the scatter step: a push with its range reduction -- which also takes the
next snapshot inside a host chunk -- or a single-workgroup launch, timed live
with HIP events on the solve stream)
and the FP64 CPU oracle timed on a bounded sample of the same queries.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "diffusion solves/s + HBM GB/s at fixed ε (batched vs plain); p50/p99 latency"
PEAK_HBM_GBS = 8000.0
CALIB_BYTES = 2 << 30
EPS_C2 = (1e-4, 1e-5, 1e-6, 1e-7)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(ops, pushes, vsize=4):
    """Algorithmic HBM bytes of a LocalGD solve: per traversed edge the column
    index and the residual read-modify-write; per pushed node its row pointers,
    the residual snapshot and reset and the x read-modify-write."""
    idx = 4
    return (idx + 2 * vsize) * ops + (2 * idx + 4 * vsize) * pushes


def push_alg_bytes(edges, entries, vsize=4):
    """Algorithmic bytes of the push kernel: per edge the column index and the
    residual read-modify-write; per work-list entry its row start, edge offset
    and scatter value."""
    return (4 + 2 * vsize) * edges + (8 + vsize) * entries


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2410_21634_amd", "csrc", "gde_kernels.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(entry_name):
    """HBM traffic per launch from a committed rocprofv3 --pmc summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "push_traffic_c2.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get(entry_name)


def pmc_summary(fetch_dir, write_dir, out_path):
    """HBM traffic per push launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of `bench.py --phase plain --copy-calib`, each
    scaled by what the same counter read for the calibration kernel (a 2 GiB
    elementwise multiply: CALIB_BYTES read and CALIB_BYTES written)."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
        return rows

    # one scatter step = one push launch with its range reduction, or one
    # single-workgroup launch (what the HIP-event timing of bench.py brackets)
    res = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = load(d, counter)
        calib = [v for k, v in rows if "MulFunctor" in k]
        push = [v for k, v in rows if "k_push<" in k]
        red = [v for k, v in rows if "k_reduce<" in k]
        small = [v for k, v in rows if "k_small<" in k]
        if not calib or not push:
            raise SystemExit(f"{d}: no calibration or push dispatches with {counter}")
        factor = CALIB_BYTES / max(calib)
        steps = len(push) + len(small)
        res[key] = dict(counter=counter, calib_counted_bytes=max(calib), factor=factor, push_launches=len(push),
                        reduce_launches=len(red), small_launches=len(small),
                        bytes_per_launch=factor * (sum(push) + sum(red) + sum(small)) / steps)
    out = dict(kernel="k_push<float,0|2> + k_reduce + k_small (scatter step)",
               workload="ppr-plain-n1M (bench.py --phase plain)",
               kernel_source_sha=kernel_source_hash(),
               bytes_per_launch=round(res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"], 1),
               fetch=res["fetch"], write=res["write"])
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def cpu_baseline_c2(G, seeds, budget_s=20.0):
    """The FP64 oracle (LocalGD and LocalCH, as it stands) on a bounded sample of
    the same queries, seeds spread over a thread pool (ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import solvers as O

    O._load()
    cores = max(1, min(16, os.cpu_count() or 1))
    solvers = {"gd": lambda eps, s: O.localgd(G.row_ptr, G.col_idx, O.PPR, 0.1, eps, [s]),
               "ch": lambda eps, s: O.localch(G.row_ptr, G.col_idx, O.PPR, 0.1, eps, [s])}
    per = {}
    for m, fn in solvers.items():
        for eps in EPS_C2:
            deadline = time.perf_counter() + budget_s / (2 * len(EPS_C2))
            done = 0
            t0 = time.perf_counter()
            with ThreadPoolExecutor(cores) as ex:
                it = iter(seeds)
                # keep `cores` solves in flight until this (method, eps) budget is spent
                futs = [ex.submit(fn, eps, int(s)) for s in (next(it, None) for _ in range(cores)) if s is not None]
                while futs:
                    futs.pop(0).result()
                    done += 1
                    if time.perf_counter() < deadline:
                        s = next(it, None)
                        if s is not None:
                            futs.append(ex.submit(fn, eps, int(s)))
            per[(m, eps)] = (done, time.perf_counter() - t0)
    # CPU time of one step (every method x eps x seed) = sum of len(seeds) / throughput
    step_s = sum(len(seeds) * dt / done for done, dt in per.values())
    return dict(value=len(seeds) * len(per) / step_s, unit="solves/s", cores=cores, kind="oracle",
                sample=("FP64 LocalGD and LocalCH oracle, PPR alpha=0.1, same graph and seeds; "
                        + ", ".join(f"{m}@{e:g}: {d} solves in {t:.1f}s" for (m, e), (d, t) in per.items())
                        + f"; {cores} threads, one solve per thread; rate of the full {len(seeds) * len(per)}-solve step mix"))


def run_c2(args):
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    t0 = time.perf_counter()
    G = W.chung_lu(1_000_000, 10_000_000, 2.5, seed=42)
    seeds = W.uniform_seeds(G, 64, seed=42)
    log(f"graph {G.summary()} built in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ctx = gde.Context(0)
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float32, device=dev)
    methods = ("gd", "ch")
    queries = [(m, eps, int(s)) for m in methods for eps in EPS_C2 for s in seeds]
    params = {(m, eps): gde.make_params("ppr", m, alpha=0.1, eps=eps, value_type=gde.F32)
              for m in methods for eps in EPS_C2}

    def step(record=None):
        # the scatter launches of every profile_every-th solve are timed with HIP
        # events (a uniform sample of the step, so that event records do not
        # slow the step they measure)
        for k, (m, eps, s) in enumerate(queries):
            timed = record is not None and k % args.profile_every == 0
            if timed:
                ctx.profile(True, reset=False)
            t = time.perf_counter()
            r = gde.solve(ctx, g, params[(m, eps)], [s], out=(oi, ov))
            if record is not None:
                record.append((m, eps, s, time.perf_counter() - t, r.iters, r.ops, r.pushes, r.status))
            if timed:
                ctx.profile(False, reset=False)

    if args.phase == "batch":  # profiling aid: only the batched call below
        queries_run = [q for q in queries if q[0] == "gd"][:1]
    else:
        queries_run = queries
    for i in range(args.warmup if args.phase != "batch" else 0):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.profile(False, reset=True)
    recs = []
    t_start = time.perf_counter()
    for i in range(args.steps if args.phase != "batch" else 0):
        step(recs)
        log(f"timed step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = ctx.profile(False, reset=True)
    if args.phase == "batch":
        for m, eps, s in queries_run:
            t = time.perf_counter()
            r = gde.solve(ctx, g, params[(m, eps)], [s], out=(oi, ov))
            recs.append((m, eps, s, time.perf_counter() - t, r.iters, r.ops, r.pushes, r.status))
        elapsed = max(elapsed, 1e-9)

    # batched comparison: the same LocalGD queries of one step as one gde_solve_batch call
    batched = None
    if not args.no_batch and args.phase != "plain":
        gd_q = [(eps, s) for m, eps, s in queries if m == "gd"]
        bparams = [params[("gd", eps)] for eps, _ in gd_q]
        bseeds = [([s], None) for _, s in gd_q]
        sched = args.schedule
        bcap = G.n // 4
        bout = (torch.empty(len(gd_q) * bcap, dtype=torch.int32, device=dev),
                torch.empty(len(gd_q) * bcap, dtype=torch.float32, device=dev))
        for _ in range(max(1, args.warmup)):
            gde.solve_batch(ctx, g, bparams, bseeds, schedule=sched, out=bout)
        torch.cuda.synchronize()
        ctx.profile(True, reset=True)
        tb = time.perf_counter()
        for _ in range(args.steps):
            bres = gde.solve_batch(ctx, g, bparams, bseeds, schedule=sched, out=bout)
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb
        bprof = ctx.profile(False, reset=True)
        plain_gd = [r for r in recs if r[0] == "gd"]
        plain_gd_rate = len(plain_gd) / sum(r[3] for r in plain_gd)
        bops = int(bres.ops.sum())
        bpush = int(bres.pushes.sum())
        batched = dict(queries=len(gd_q), solves_per_s=round(len(gd_q) * args.steps / tb, 2),
                       ms_per_batch=round(1e3 * tb / args.steps, 3),
                       plain_solves_per_s_same_queries=round(plain_gd_rate, 2),
                       speedup_vs_plain=round(len(gd_q) * args.steps / tb / plain_gd_rate, 2),
                       hbm_gbs_alg=round(alg_bytes(bops, bpush) * args.steps / tb / 1e9, 2),
                       kernel_ms=round(bprof["batch_ms"] / max(bprof["batch_launches"], 1), 3),
                       lane_edges_per_batch=int(bprof["batch_lane_edges"] // max(args.steps, 1)),
                       entries_per_batch=int(bprof["batch_entries"] // max(args.steps, 1)),
                       schedule=sched or "default", not_converged=int((bres.status != 0).sum()))
        log(f"batched: {batched}")

    nq = len(queries)
    ms_per_step = 1e3 * elapsed / args.steps
    value = nq * args.steps / elapsed
    lat = np.array([r[3] for r in recs]) * 1e3
    ops = sum(r[5] for r in recs)
    pushes = sum(r[6] for r in recs)
    gbs = alg_bytes(ops, pushes) / elapsed / 1e9
    per = {}
    for m in methods:
        for eps in EPS_C2:
            sel = [r for r in recs if r[0] == m and r[1] == eps]
            if not sel:  # --phase batch times one plain query only
                continue
            per[f"{m}@{eps:g}"] = dict(
                solves_per_s=len(sel) / sum(r[3] for r in sel), p50_ms=float(np.percentile([r[3] * 1e3 for r in sel], 50)),
                mean_iters=float(np.mean([r[4] for r in sel])), mean_ops=float(np.mean([r[5] for r in sel])),
                not_converged=int(sum(r[7] != 0 for r in sel)))
    # roofline of the push kernel, from the live event timing of the timed region
    launches = max(prof["launches"], 1)
    pb = push_alg_bytes(prof["edges"], prof["entries"])
    avg_ms = prof["total_ms"] / launches
    achieved = pb / (prof["total_ms"] * 1e-3) / 1e9 if prof["total_ms"] > 0 else 0.0
    traffic = traffic_from_profile("bytes_per_launch")
    roof = dict(bound="hbm", achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 5), traffic=traffic, kernel="scatter step: k_push + k_reduce, or k_small",
                launches=prof["launches"], avg_launch_us=round(avg_ms * 1e3, 3),
                alg_bytes_per_launch=round(pb / launches, 1),
                timed_launches=f"scatter launches of every {args.profile_every}th solve of the timed steps")
    out = dict(
        metric=METRIC, value=round(value, 3), unit="solves/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms_per_step, 3), higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload="ppr-plain-n1M: Chung-Lu n=1e6, 1e7 edges, gamma 2.5, seed 42; 64 seeds x eps "
                             "{1e-4,1e-5,1e-6,1e-7} x {LocalGD, LocalCH}, PPR alpha 0.1, one solve at a time",
                    n=G.n, edges=G.nnz // 2, d_max=int(G.degrees.max()), solves_per_step=nq, path="plain"),
        hbm_gbs_alg=round(gbs, 2), hbm_frac_alg=round(gbs / PEAK_HBM_GBS, 5),
        latency_ms=dict(p50=round(float(np.percentile(lat, 50)), 4), p99=round(float(np.percentile(lat, 99)), 4)),
        per_query=per, roofline=roof, batched=batched)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_c2(G, seeds, budget_s=args.cpu_budget)
    g.close()
    ctx.close()
    return out


def build_graph_device(W, n, E, gamma, seed, gde, ctx, torch):
    t0 = time.perf_counter()
    G = W.chung_lu(n, E, gamma, seed=seed)
    log(f"graph {G.summary()} built in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    return G, gde.Graph(ctx, rp, ci), (rp, ci)


def run_c4(args):
    """Batched: 1,024 degree-stratified seeds, eps log-uniform in [1e-7, 1e-4], PPR
    alpha 0.1, on the n = 10^7, 2e8-edge, gamma 2.2 graph; one gde_solve_batch call
    against the same queries solved one at a time (the plain path, on a sample)."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    ctx = gde.Context(0)
    G, g, keep = build_graph_device(W, 10_000_000, 200_000_000, 2.2, 42, gde, ctx, torch)
    B = 1024
    seeds = W.stratified_seeds(G, B, bins=16, seed=42)
    eps = W.log_uniform_eps(B, 1e-7, 1e-4, seed=42)
    params = [gde.make_params("ppr", alpha=0.1, eps=float(e), value_type=gde.F32) for e in eps]
    bseeds = [([int(s)], None) for s in seeds]
    cap = 2_000_000
    dev = torch.device("cuda:0")
    bout = (torch.empty(B * cap, dtype=torch.int32, device=dev), torch.empty(B * cap, dtype=torch.float32, device=dev))
    for i in range(args.warmup):
        gde.solve_batch(ctx, g, params, bseeds, schedule=args.schedule, out=bout)
        log(f"warmup batch {i + 1} done")
    torch.cuda.synchronize()
    ctx.profile(True, reset=True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = gde.solve_batch(ctx, g, params, bseeds, schedule=args.schedule, out=bout)
        log(f"timed batch {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile(False, reset=True)
    ops = int(res.ops.sum())
    pushes = int(res.pushes.sum())
    value = B * args.steps / el
    gbs = alg_bytes(ops, pushes) * args.steps / el / 1e9
    kms = prof["batch_ms"] / max(prof["batch_launches"], 1)
    # batched kernel roofline: per (edge, query) update 12 B, per (query, node) push 24 B
    kb = alg_bytes(ops, pushes) / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    # the plain path on a stratified sample of the same queries (one at a time)
    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float32, device=dev)
    samp = list(range(0, B, max(1, B // args.plain_sample)))
    gde.solve(ctx, g, params[samp[0]], [int(seeds[samp[0]])], out=(oi, ov))
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for j in samp:
        gde.solve(ctx, g, params[j], [int(seeds[j])], out=(oi, ov))
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    plain_rate = len(samp) / tp
    out = dict(metric=METRIC, value=round(value, 2), unit="solves/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(1e3 * el / args.steps, 3), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="ppr-batched-n10M: Chung-Lu n=1e7, 2e8 edges, gamma 2.2, seed 42; 1,024 "
                                    "degree-stratified seeds, eps log-uniform [1e-7,1e-4], PPR alpha 0.1, one "
                                    "gde_solve_batch call", n=G.n, edges=G.nnz // 2, queries=B, path="batched",
                           schedule=args.schedule or "default"),
               hbm_gbs_alg=round(gbs, 2), hbm_frac_alg=round(gbs / PEAK_HBM_GBS, 5),
               roofline=dict(bound="hbm", achieved=round(kb, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                             frac=round(kb / PEAK_HBM_GBS, 5), traffic=None,
                             kernel="batched snap+push launches (whole solve)", kernel_ms=round(kms, 3)),
               plain=dict(sample=len(samp), solves_per_s=round(plain_rate, 2),
                          batched_speedup=round(value / plain_rate, 2)),
               stats=dict(total_edge_updates=int(ops), total_pushes=int(pushes),
                          not_converged=int((res.status != 0).sum()), mean_iters=float(res.iters.mean())))
    g.close()
    ctx.close()
    return out


def run_serve(args):
    """Serving: open-loop Poisson arrivals of mixed PPR / Katz / HK queries (half
    single seeds, half 8-node seed sets, eps log-uniform [1e-7, 1e-4]) with a
    10,000-edge insert batch every 100 ms, swept over arrival rates.  Queries and
    insert batches are drawn before the clock starts; latency is completion time
    minus scheduled arrival time."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    ctx = gde.Context(0)
    n, E = (10_000_000, 200_000_000) if not args.small else (1_000_000, 10_000_000)
    G, g, keep = build_graph_device(W, n, E, 2.2, 42, gde, ctx, torch)
    lo, hi = g.lambda_max(max_iters=300, rtol=1e-3)
    beta = 0.5 / hi
    log(f"lambda bounds [{lo:.3f}, {hi:.3f}], beta {beta:.4g}")
    total_s = args.warm_s + args.serve_s
    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    existing = set()
    inserts = [W.insert_batch(G, args.insert_k, rng, existing) for _ in range(int(total_s / 0.1))]
    log(f"{len(inserts)} insert batches of {args.insert_k} drawn in {time.perf_counter() - t0:.1f}s")
    pool = W.stratified_seeds(G, 4096, bins=16, seed=7)
    sets = [W.seed_set(G, int(a), 8, rng) for a in pool[::4]]
    results = []
    for qps in args.qps:
        arr = W.poisson_arrivals(qps, total_s, seed=int(qps))
        qs = []
        for _ in range(len(arr)):
            kind = ("ppr", "katz", "hk")[int(rng.integers(0, 3))]
            e = float(10 ** rng.uniform(-7, -4))
            if rng.random() < 0.5:
                idx, val = np.array([pool[int(rng.integers(0, len(pool)))]], np.int32), np.ones(1)
            else:
                idx, val = sets[int(rng.integers(0, len(sets)))]
            if kind == "ppr":
                p = gde.make_params("ppr", alpha=0.1, eps=e)
            elif kind == "katz":
                p = gde.make_params("katz", beta=beta, eps=max(e, 1e-6), lambda_bound=hi)
            else:
                p = gde.make_params("hk", tau=5.0, K=30, eps=max(e, 1e-6))
            qs.append((p, idx, val, kind))
        srv = gde.Server(ctx, g, lanes_per_group=16, max_groups=args.groups, iters_per_step=args.iters_per_step,
                         result_capacity=2_000_000)
        lat, sub_at, sub_kind = [], {}, {}
        kinds = {k: [0, 0, []] for k in ("ppr", "katz", "hk")}  # completed, submitted, latencies
        submitted = completed = i = ins = 0
        t0 = time.perf_counter()
        deadline = total_s + 2.0
        while True:
            now = time.perf_counter() - t0
            if now > deadline:
                break
            # at most 256 submissions per pass, so that a client that cannot keep up
            # with the arrival schedule still polls (its lag counts as latency)
            burst = 0
            while i < len(arr) and arr[i] <= now and burst < 256:
                burst += 1
                t = srv.submit(*qs[i][:3])
                sub_at[t] = arr[i]
                sub_kind[t] = qs[i][3]
                submitted += arr[i] >= args.warm_s
                kinds[qs[i][3]][1] += int(arr[i] >= args.warm_s)
                i += 1
            while ins < len(inserts) and (ins + 1) * 0.1 <= now:
                srv.insert_edges(*inserts[ins])
                ins += 1
            done = srv.poll()
            tn = time.perf_counter() - t0
            for c in done:
                t_arr = sub_at.pop(c["ticket"])
                kd = kinds[sub_kind.pop(c["ticket"])]
                if t_arr >= args.warm_s:
                    lat.append(tn - t_arr)
                    completed += 1
                    kd[0] += 1
                    kd[2].append((tn - t_arr) * 1e3)
            if i >= len(arr) and not sub_at:
                break
        srv.close()
        lat_ms = np.array(lat) * 1e3
        rec = dict(qps=qps, submitted=int(submitted), completed=int(completed),
                   offered=int(np.sum(arr >= args.warm_s)),
                   completion_ratio=round(completed / max(int(np.sum(arr >= args.warm_s)), 1), 4),
                   solves_per_s=round(completed / args.serve_s, 2), inserted_edges=ins * args.insert_k,
                   p50_ms=round(float(np.percentile(lat_ms, 50)), 3) if len(lat_ms) else None,
                   p99_ms=round(float(np.percentile(lat_ms, 99)), 3) if len(lat_ms) else None,
                   by_kind={k: dict(completed=int(v[0]), submitted=int(v[1]),
                                    p50_ms=round(float(np.percentile(v[2], 50)), 3) if v[2] else None,
                                    p99_ms=round(float(np.percentile(v[2], 99)), 3) if v[2] else None)
                            for k, v in kinds.items()})
        log(f"serve {rec}")
        results.append(rec)
    ok = [r for r in results if r["completion_ratio"] >= 0.99]
    stated = max(ok, key=lambda r: r["qps"]) if ok else results[0]
    out = dict(metric=METRIC, value=stated["solves_per_s"], unit="solves/s", n_gpus=1, steps=len(results),
               warmup=0, ms_per_step=None, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=f"serving: Chung-Lu n={n}, {E} edges, gamma 2.2; Poisson arrivals of mixed "
                                    f"PPR/Katz/HK, {args.insert_k}-edge inserts every 100 ms",
                           stated_qps=stated["qps"], serve_s=args.serve_s, warm_s=args.warm_s),
               latency_ms=dict(p50=stated["p50_ms"], p99=stated["p99_ms"]), sweep=results)
    g.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c2", "c4", "serve"])
    ap.add_argument("--plain-sample", type=int, default=64, help="c4: plain solves timed for the comparison")
    ap.add_argument("--qps", type=float, nargs="+", default=[1000, 2000, 5000, 10000, 20000, 50000])
    ap.add_argument("--warm-s", type=float, default=2.0)
    ap.add_argument("--serve-s", type=float, default=10.0)
    ap.add_argument("--insert-k", type=int, default=10000)
    ap.add_argument("--groups", type=int, default=16)
    ap.add_argument("--iters-per-step", type=int, default=4)
    ap.add_argument("--small", action="store_true", help="serve: the n=1e6 graph instead of n=1e7")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--phase", default="all", choices=["all", "plain", "batch"],
                    help="profiling aid: run only one path (the JSON line then covers that path only)")
    ap.add_argument("--schedule", default=None, help='batched schedule JSON, e.g. {"lanes":16}')
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="write the per-launch push traffic from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time the scatter launches of every k-th plain solve with HIP events")
    ap.add_argument("--copy-calib", action="store_true",
                    help="end with one 256 MiB device-to-device copy kernel, the calibration for HBM byte counters")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print(json.dumps(dict(error="bench.py measures one GPU only; multi-GPU sharding is by query "
                                    "(replicated graph) and is described, not run")), flush=True)
        sys.exit(2)
    out = {"c2": run_c2, "c4": run_c4, "serve": run_serve}[args.workload](args)
    print(json.dumps(out), flush=True)
    if args.copy_calib:
        import torch

        # 2 GiB each way, far beyond the caches: one elementwise kernel that reads
        # CALIB_BYTES and writes CALIB_BYTES, the reference for the byte counters
        a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log(f"copy calibration: {CALIB_BYTES} bytes read, {CALIB_BYTES} bytes written")


if __name__ == "__main__":
    main()
