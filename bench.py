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
(the push / residual scatter, timed live with HIP events on the solve stream)
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


def cpu_baseline_c2(G, seeds, budget_s=20.0):
    """The FP64 oracle (LocalGD, as it stands) on a bounded sample of the same
    queries, seeds spread over a thread pool (ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import solvers as O

    O._load()
    cores = max(1, min(16, os.cpu_count() or 1))
    per_eps = {}
    for eps in EPS_C2:
        deadline = time.perf_counter() + budget_s / len(EPS_C2)
        done = 0
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            futs = []
            it = iter(seeds)
            # keep `cores` solves in flight until the per-eps budget is spent
            for _ in range(cores):
                s = next(it, None)
                if s is not None:
                    futs.append(ex.submit(O.localgd, G.row_ptr, G.col_idx, O.PPR, 0.1, eps, [int(s)]))
            while futs:
                f = futs.pop(0)
                f.result()
                done += 1
                if time.perf_counter() < deadline:
                    s = next(it, None)
                    if s is not None:
                        futs.append(ex.submit(O.localgd, G.row_ptr, G.col_idx, O.PPR, 0.1, eps, [int(s)]))
        dt = time.perf_counter() - t0
        per_eps[eps] = (done, dt)
    # CPU time of one step's LocalGD queries = sum over eps of len(seeds) / throughput(eps)
    step_s = sum(len(seeds) * dt / done for done, dt in per_eps.values())
    return dict(value=len(seeds) * len(EPS_C2) / step_s, unit="solves/s", cores=cores, kind="oracle",
                sample=("FP64 LocalGD oracle, PPR alpha=0.1, same graph and seeds; per eps "
                        + ", ".join(f"{e:g}: {d} solves in {t:.1f}s" for e, (d, t) in per_eps.items())
                        + f"; {cores} threads, one solve per thread; throughput of the 4-eps LocalGD mix"))


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
        for m, eps, s in queries:
            t = time.perf_counter()
            r = gde.solve(ctx, g, params[(m, eps)], [s], out=(oi, ov))
            if record is not None:
                record.append((m, eps, s, time.perf_counter() - t, r.iters, r.ops, r.pushes, r.status))

    if args.phase == "batch":  # profiling aid: only the batched call below
        queries_run = [q for q in queries if q[0] == "gd"][:1]
    else:
        queries_run = queries
    for i in range(args.warmup if args.phase != "batch" else 0):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.profile(True, reset=True)
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
        bops = sum(r.ops for r in bres)
        bpush = sum(r.pushes for r in bres)
        batched = dict(queries=len(gd_q), solves_per_s=round(len(gd_q) * args.steps / tb, 2),
                       ms_per_batch=round(1e3 * tb / args.steps, 3),
                       plain_solves_per_s_same_queries=round(plain_gd_rate, 2),
                       speedup_vs_plain=round(len(gd_q) * args.steps / tb / plain_gd_rate, 2),
                       hbm_gbs_alg=round(alg_bytes(bops, bpush) * args.steps / tb / 1e9, 2),
                       kernel_ms=round(bprof["batch_ms"] / max(bprof["batch_launches"], 1), 3),
                       schedule=sched or "default", not_converged=int(sum(r.status != 0 for r in bres)))
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
                frac=round(achieved / PEAK_HBM_GBS, 5), traffic=traffic, kernel="k_push<float,0|2> (residual scatter)",
                launches=prof["launches"], avg_launch_us=round(avg_ms * 1e3, 3),
                alg_bytes_per_launch=round(pb / launches, 1))
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c2"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--phase", default="all", choices=["all", "plain", "batch"],
                    help="profiling aid: run only one path (the JSON line then covers that path only)")
    ap.add_argument("--schedule", default=None, help='batched schedule JSON, e.g. {"lanes":16}')
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps(dict(error="this build measures one GPU only; multi-GPU sharding is by query "
                                    "(replicated graph) and is described, not run")), flush=True)
        sys.exit(2)
    out = run_c2(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
