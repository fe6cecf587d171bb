#!/usr/bin/env python3
"""Throughput of the local diffusion solvers on one MI355X.

Default workload (the batched configuration on the n = 10^7 power-law graph):
undirected Chung-Lu graph, n = 10,000,000, 200,000,000 edges (nnz 4e8), degree
exponent 2.2, RNG seed 42, int32 CSR, FP32 x / r.  One step = ONE
gde_solve_batch call over 1,024 PPR queries (alpha 0.1, LocalGD): seeds
degree-stratified over 16 log2-spaced degree bins, eps log-uniform in
[1e-7, 1e-4]; inputs and outputs stay in HBM.  The same 1,024 queries are also
solved one at a time (the plain path) for the batched/plain ratio.

Printed: one JSON line with solves/s of the batched step (value), the
algorithmic HBM GB/s of the whole batch, the roofline of its dominant kernel
(the batched push, each launch timed live with HIP events on the solve stream),
the FP64 CPU oracle timed on a bounded, eps-stratified sample of the same
queries, and sub-records for the other configurations: the plain 512-solve
mix on the n = 10^6 graph, the n = 10^4 FP64 latency, Katz and heat-kernel
throughput on the n = 2.4 * 10^6 graph, and a short serving run on the n = 10^7
graph with edge insertions.
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


def kernel_source_hash(source="gde_kernels.hip"):
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2410_21634_amd", "csrc", source), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(fname, source, entry_name, kernel_names=None):
    """HBM traffic per launch from a committed rocprofv3 --pmc summary
    (profiles/<fname>), if it was taken on the current kernel source (and, when
    kernel_names is given, on exactly those kernel instantiations)."""
    path = os.path.join(ROOT, "profiles", fname)
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash(source):
        return None
    if kernel_names is not None and sorted(d.get("kernel_names", [])) != sorted(kernel_names):
        return None
    return d.get(entry_name)


# --pmc-summary targets: which dispatches make up one timed launch of the
# roofline kernel, its source file, and where the summary is kept
PMC_TARGETS = {
    "plain": dict(source="gde_kernels.hip", out="push_traffic_c2.json",
                  kernel="k_push<float,0|2> + k_reduce + k_small (scatter step)",
                  workload="ppr-plain-n1M (bench.py --workload c2 --phase plain)",
                  step=("k_push<", "k_small<"), extra=("k_reduce<",)),
    "batch": dict(source="gde_batch_kernels.hip", out="batch_push_traffic_c4_L{lanes}.json",
                  kernel="k_batch_push<float,L,true> (batched residual scatter)",
                  workload="ppr-batched-n10M (bench.py --workload c4 --no-sub --no-cpu-baseline --steps 2 "
                           "--warmup 1 --schedule <the chosen lanes> --copy-calib)",
                  step=("k_batch_push<",), extra=()),
}


def pmc_summary(target, fetch_dir, write_dir):
    """HBM traffic per timed launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of a bench run ending with --copy-calib, each
    scaled by what the same counter read for the calibration kernel (a 2 GiB
    elementwise multiply: CALIB_BYTES read and CALIB_BYTES written)."""
    import csv
    import glob

    tg = PMC_TARGETS[target]

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
        return rows

    res = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = load(d, counter)
        calib = [v for k, v in rows if "MulFunctor" in k]
        step = [v for k, v in rows if any(m in k for m in tg["step"])]
        names = sorted({k.split("(")[0].replace("void ", "").strip() for k, _ in rows
                        if any(m in k for m in tg["step"])})
        extra = [v for k, v in rows if any(m in k for m in tg["extra"])]
        if not calib or not step:
            raise SystemExit(f"{d}: no calibration or timed dispatches with {counter}")
        factor = CALIB_BYTES / max(calib)
        res[key] = dict(counter=counter, calib_counted_bytes=max(calib), factor=factor, launches=len(step),
                        extra_dispatches=len(extra), bytes_per_launch=factor * (sum(step) + sum(extra)) / len(step),
                        kernel_names=names)
    out = dict(kernel=tg["kernel"], workload=tg["workload"], kernel_source_sha=kernel_source_hash(tg["source"]),
               kernel_names=res["fetch"]["kernel_names"],
               bytes_per_launch=round(res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"], 1),
               fetch=res["fetch"], write=res["write"])
    lanes = ""
    if "{lanes}" in tg["out"]:  # one summary per lane width: the name carries it
        import re
        m = {re.search(r"<float, (\d+),", k).group(1) for k in out["kernel_names"]}
        if len(m) != 1:
            raise SystemExit(f"expected one lane width among {out['kernel_names']}")
        lanes = m.pop()
    with open(os.path.join(ROOT, "profiles", tg["out"].format(lanes=lanes)), "w") as fh:
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
        bparams = gde.params_array([params[("gd", eps)] for eps, _ in gd_q])
        bseeds = np.array([s for _, s in gd_q], dtype=np.int32)  # one seed node per query
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
        # the LocalCH queries of the step as one batch as well (batched LocalCH)
        ch_q = [(eps, s) for m, eps, s in queries if m == "ch"]
        if ch_q:
            cparams = gde.params_array([params[("ch", eps)] for eps, _ in ch_q])
            cseeds = np.array([s for _, s in ch_q], dtype=np.int32)
            del bout
            # LocalCH's support can exceed n/4 at small eps: a full-length buffer per query
            cout = (torch.empty(len(ch_q) * G.n, dtype=torch.int32, device=dev),
                    torch.empty(len(ch_q) * G.n, dtype=torch.float32, device=dev))
            gde.solve_batch(ctx, g, cparams, cseeds, schedule=sched, out=cout)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            for _ in range(args.steps):
                cres = gde.solve_batch(ctx, g, cparams, cseeds, schedule=sched, out=cout)
            torch.cuda.synchronize()
            tc = time.perf_counter() - tc
            plain_ch = [r for r in recs if r[0] == "ch"]
            plain_ch_rate = len(plain_ch) / sum(r[3] for r in plain_ch)
            batched["localch"] = dict(queries=len(ch_q), solves_per_s=round(len(ch_q) * args.steps / tc, 2),
                                      plain_solves_per_s_same_queries=round(plain_ch_rate, 2),
                                      speedup_vs_plain=round(len(ch_q) * args.steps / tc / plain_ch_rate, 2),
                                      not_converged=int((cres.status != 0).sum()))
            del cout
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
    traffic = traffic_from_profile("push_traffic_c2.json", "gde_kernels.hip", "bytes_per_launch")
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


def host_cpu():
    """CPU model and logical core count of this host (for the baseline record)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline_c4(G, seeds, eps, budget_s=30.0, threads=16):
    """The FP64 LocalGD oracle, as it stands, on the batched queries: (1) every
    query of the batch spread over a thread pool, one single-threaded solve per
    thread (ctypes releases the GIL), and (2) one solve at a time on one core,
    median latency over every 16th query in eps order.  The pool is capped at the
    host CPU share of one GPU (16 threads)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import solvers as O

    O._load()
    model, ncpu = host_cpu()
    cores = max(1, min(threads, ncpu))
    order = np.argsort(eps, kind="stable")
    rp64 = G.row_ptr.astype(np.int64)

    def one(i):
        t = time.perf_counter()
        O.localgd(rp64, G.col_idx, O.PPR, 0.1, float(eps[i]), [int(seeds[i])])
        return time.perf_counter() - t

    t1 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        done = len(list(ex.map(one, range(len(seeds)))))
    wall = time.perf_counter() - t1
    lat = []
    t0 = time.perf_counter()
    for i in order[8::16]:
        lat.append(one(int(i)))
        if time.perf_counter() - t0 > budget_s:
            break
    return dict(value=round(done / wall, 3), unit="solves/s", cores=cores, kind="oracle",
                host_cpu=model, host_logical_cpus=ncpu,
                latency_1core_ms=dict(median=round(1e3 * float(np.median(lat)), 3),
                                      p99=round(1e3 * float(np.percentile(lat, 99)), 3), solves=len(lat)),
                sample=(f"FP64 LocalGD oracle, PPR alpha=0.1, same n=1e7 graph: all {done} queries of the batch on "
                        f"{cores} threads, one single-threaded solve per thread, in {wall:.1f}s; 1-core latency over "
                        f"{len(lat)} queries (every 16th in eps order)"))


def c4_inputs(W):
    t0 = time.perf_counter()
    G = W.chung_lu(10_000_000, 200_000_000, 2.2, seed=42)
    log(f"graph {G.summary()} built in {time.perf_counter() - t0:.1f}s")
    B = 1024
    seeds = W.stratified_seeds(G, B, bins=16, seed=42)
    eps = W.log_uniform_eps(B, 1e-7, 1e-4, seed=42)
    return G, seeds, eps


# returning FP32 atomic adds to random words of a 16 GB array, 2^28 updates from
# 1M threads, measured on MI355X (16.5 G/s; 20.9 G/s when the array is 32 MB)
RANDOM_ATOMIC_RATE = 16.5e9


def batch_push_bytes(prof, vsize=4):
    """Algorithmic bytes of the batched push launches (the batched rule): the
    column indices of every distinct CSR row pushed in a round, once, whatever
    the number of queries pushing it; per (edge, query) update the residual
    read-modify-write."""
    return 4 * prof["batch_row_vol"] + 2 * vsize * prof["batch_lane_edges"]


def batch_alg_bytes(prof, lane_pushes, vsize=4):
    """Algorithmic bytes of whole batched solves: the push bytes above, plus per
    distinct row and round its row pointers, plus per (node, query) push the
    residual snapshot and reset and the x read-modify-write."""
    return batch_push_bytes(prof, vsize) + 8 * prof["batch_rows"] + 4 * vsize * lane_pushes


def run_c4(args):
    """Batched: 1,024 degree-stratified seeds, eps log-uniform in [1e-7, 1e-4], PPR
    alpha 0.1, on the n = 10^7, 2e8-edge, gamma 2.2 graph; one gde_solve_batch call
    per step, against the same queries solved one at a time (the plain path)."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    G, seeds, eps = c4_inputs(W)
    B = len(seeds)
    ctx = gde.Context(0)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    params = [gde.make_params("ppr", alpha=0.1, eps=float(e), value_type=gde.F32) for e in eps]
    bparams = gde.params_array(params)  # built once: the calls only marshal
    bseeds = np.asarray(seeds, dtype=np.int32)  # one seed node per query
    cap = 2_000_000
    bout = (torch.empty(B * cap, dtype=torch.int32, device=dev), torch.empty(B * cap, dtype=torch.float32, device=dev))
    for i in range(args.warmup):
        gde.solve_batch(ctx, g, bparams, bseeds, schedule=args.schedule, out=bout)
        log(f"warmup batch {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.profile(True, reset=True)
    t0 = time.perf_counter()
    per_batch = []
    for i in range(args.steps):
        tb = time.perf_counter()
        res = gde.solve_batch(ctx, g, bparams, bseeds, schedule=args.schedule, out=bout)  # returns when done
        per_batch.append(time.perf_counter() - tb)
        log(f"timed batch {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile(False, reset=True)
    tuned = ctx.batch_tuned(g, "ppr", gde.F32, B)
    lanes = tuned[0] if tuned else json.loads(args.schedule or "{}").get("lanes", 16)
    ops = int(res.ops.sum())
    pushes = int(res.pushes.sum())
    value = B * args.steps / el
    K = max(args.steps, 1)
    whole = batch_alg_bytes(prof, pushes * K) / K  # per batch
    gbs = whole * args.steps / el / 1e9
    pl = max(prof["batch_push_launches"], 1)
    push_ms = prof["batch_push_ms"] / pl
    push_bytes = batch_push_bytes(prof) / pl
    achieved = push_bytes / (push_ms * 1e-3) / 1e9 if push_ms > 0 else 0.0
    # counters count only if they were taken on this lane width's push kernel
    traffic = traffic_from_profile(f"batch_push_traffic_c4_L{lanes}.json", "gde_batch_kernels.hip", "bytes_per_launch",
                                   kernel_names=[f"gde::k_batch_push<float, {lanes}, true>"])
    roof = dict(bound="hbm", achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 5), traffic=traffic,
                kernel=f"k_batch_push<float,{lanes},true> (batched residual scatter)", launches=prof["batch_push_launches"],
                avg_launch_us=round(push_ms * 1e3, 3), alg_bytes_per_launch=round(push_bytes, 1),
                timed_launches="every push launch of the timed batches, HIP events on the solve stream",
                byte_rule="4 B per column index of each distinct row pushed in a round + 8 B per (edge, query) "
                          "residual read-modify-write")
    # what bounds it: one memory-side atomic per (edge, query), against the rate of
    # returning FP32 atomics to random words of a 16 GB array measured on MI355X
    rate = prof["batch_lane_edges"] / pl / (push_ms * 1e-3) if push_ms > 0 else 0.0
    roof["update_rate"] = dict(lane_edge_atomics_per_s=round(rate), random_atomic_rate_per_s=RANDOM_ATOMIC_RATE,
                               frac=round(rate / RANDOM_ATOMIC_RATE, 4))
    kms = prof["batch_ms"] / max(prof["batch_launches"], 1)
    # the plain path on the same queries, one at a time
    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float32, device=dev)
    samp = list(range(0, B, max(1, B // args.plain_sample)))
    gde.solve(ctx, g, params[samp[0]], [int(seeds[samp[0]])], out=(oi, ov))
    torch.cuda.synchronize()
    tp = time.perf_counter()
    nconv_plain = 0
    for j in samp:
        r = gde.solve(ctx, g, params[j], [int(seeds[j])], out=(oi, ov))
        nconv_plain += int(r.status != gde.OK)
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    plain_rate = len(samp) / tp
    log(f"c4: batched {value:.1f} solves/s, plain {plain_rate:.1f} solves/s")
    out = dict(metric=METRIC, value=round(value, 2), unit="solves/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(1e3 * el / args.steps, 3), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="ppr-batched-n10M: Chung-Lu n=1e7, 2e8 edges, gamma 2.2, seed 42; 1,024 "
                                    "degree-stratified seeds (16 log2 degree bins), eps log-uniform [1e-7,1e-4] "
                                    "(seed 42), PPR alpha 0.1, LocalGD, FP32; one gde_solve_batch call per step",
                           n=G.n, edges=G.nnz // 2, d_max=int(G.degrees.max()), queries=B, path="batched",
                           schedule=args.schedule or "default",
                           schedule_chosen=dict(lanes=tuned[0], blocks_per_cu=tuned[1]) if tuned else None),
               hbm_gbs_alg=round(gbs, 2), hbm_frac_alg=round(gbs / PEAK_HBM_GBS, 5),
               roofline=roof,
               batch=dict(ms_per_batch=round(1e3 * el / args.steps, 3),
                          ms_per_batch_median=round(1e3 * float(np.median(per_batch)), 3),
                          ms_per_batch_min=round(1e3 * min(per_batch), 3), solve_span_ms=round(kms, 3),
                          push_ms_per_batch=round(prof["batch_push_ms"] / K, 3),
                          lane_edges=int(prof["batch_lane_edges"] // K), entries=int(prof["batch_entries"] // K),
                          distinct_rows=int(prof["batch_rows"] // K), distinct_row_vol=int(prof["batch_row_vol"] // K),
                          lane_pushes=pushes, alg_bytes=int(whole), not_converged=int((res.status != 0).sum()),
                          mean_iters=round(float(res.iters.mean()), 3), max_iters=int(res.iters.max())),
               plain=dict(queries=len(samp), solves_per_s=round(plain_rate, 2), not_converged=nconv_plain,
                          batched_speedup=round(value / plain_rate, 2)))
    if not args.no_sub:
        out["serving"] = run_serve_sub(args, ctx, g, G)
        out["global_gd"] = sub_global_roofline(ctx, g, G, seeds, dev)
    g.close()
    ctx.close()
    del rp, ci, bout
    torch.cuda.empty_cache()
    if not args.no_sub:
        out["sub"] = dict(c2_plain=sub_c2(args), c1_latency=sub_c1(), c3_katz_hk=sub_c3(),
                          global_vs_local=sub_global_vs_local(), dynamic=sub_dynamic(), localsor=sub_sor())
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_c4(G, seeds, eps, budget_s=args.cpu_budget)
    return out


def sub_c2(args):
    """One step of the plain 512-solve mix on the n = 10^6 graph (and the batched
    call over its LocalGD queries), as a sub-record."""
    sub_args = argparse.Namespace(**vars(args))
    sub_args.steps, sub_args.warmup, sub_args.no_cpu_baseline, sub_args.phase = 1, 1, True, "all"
    r = run_c2(sub_args)
    keep = ("value", "unit", "ms_per_step", "hbm_gbs_alg", "hbm_frac_alg", "latency_ms", "per_query", "roofline",
            "batched")
    return dict(config=r["config"], **{k: r[k] for k in keep})


def sub_c1():
    """Latency of one FP64 PPR LocalGD solve on the n = 10^4 graph (median / p99
    over 100 repeats, device outputs)."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    G = W.chung_lu(10_000, 50_000, 2.5, seed=42)
    seed = int(W.uniform_seeds(G, 1, seed=42)[0])
    ctx = gde.Context(0)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    p = gde.make_params("ppr", alpha=0.1, eps=1e-6, value_type=gde.F64)
    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float64, device=dev)
    for _ in range(3):
        r = gde.solve(ctx, g, p, [seed], out=(oi, ov))
    lat = []
    for _ in range(100):
        t = time.perf_counter()
        r = gde.solve(ctx, g, p, [seed], out=(oi, ov))
        lat.append(time.perf_counter() - t)
    g.close()
    ctx.close()
    lat = np.array(lat) * 1e6
    return dict(workload="Chung-Lu n=1e4, 5e4 edges, gamma 2.5, seed 42; one uniform seed; PPR alpha 0.1, "
                         "eps 1e-6, LocalGD, FP64", seed=seed, iters=r.iters, ops=r.ops,
                latency_us=dict(median=round(float(np.median(lat)), 2), p99=round(float(np.percentile(lat, 99)), 2)))


def sub_c3():
    """Katz (beta = 0.5 / lambda_lower) and heat kernel (tau 5, K 30) at eps 1e-6,
    32 uniform seeds, FP32, on the n = 2.4 * 10^6 graph: solves/s of each."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    t0 = time.perf_counter()
    G = W.chung_lu(2_400_000, 62_000_000, 2.3, seed=42)
    log(f"graph {G.summary()} built in {time.perf_counter() - t0:.1f}s")
    seeds = W.uniform_seeds(G, 32, seed=42)
    ctx = gde.Context(0)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    lo, hi = g.lambda_max(max_iters=300, rtol=1e-3)
    beta = 0.5 / lo
    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float32, device=dev)
    cap_b = G.n  # result entries per batched query
    out = dict(workload="Chung-Lu n=2.4e6, 6.2e7 edges, gamma 2.3, seed 42; 32 uniform seeds one by one, and 256 "
                        "uniform seeds in one batch; eps 1e-6, FP32",
               lambda_bounds=[round(lo, 4), round(hi, 4)], beta=beta)
    for name, p in (("katz", gde.make_params("katz", beta=beta, eps=1e-6, lambda_bound=hi, value_type=gde.F32)),
                    ("hk", gde.make_params("hk", tau=5.0, K=30, eps=1e-6, value_type=gde.F32))):
        gde.solve(ctx, g, p, [int(seeds[0])], out=(oi, ov))
        torch.cuda.synchronize()
        t = time.perf_counter()
        ops = 0
        for s in seeds:
            r = gde.solve(ctx, g, p, [int(s)], out=(oi, ov))
            ops += r.ops
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        out[name] = dict(solves_per_s=round(len(seeds) / t, 2), mean_ops=round(ops / len(seeds), 1))
        # the same query kind for 256 uniform seeds in one gde_solve_batch call
        # (Katz: batched LocalGD; heat kernel: the batched level push)
        bseeds = np.asarray(W.uniform_seeds(G, 256, seed=43), dtype=np.int32)
        bparams = gde.params_array([p] * 256)
        bo = (torch.empty(256 * cap_b, dtype=torch.int32, device=dev),
              torch.empty(256 * cap_b, dtype=torch.float32, device=dev))
        gde.solve_batch(ctx, g, bparams, bseeds, out=bo)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = gde.solve_batch(ctx, g, bparams, bseeds, out=bo)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        out[name].update(batched_256_solves_per_s=round(256 / t, 1), batched_mean_ops=round(float(res.ops.mean()), 1))
        log(f"c3 {name}: {out[name]}")
        del bo
    g.close()
    ctx.close()
    torch.cuda.empty_cache()
    return out


def glob_bytes_per_iter(n, nnz, vsize):
    """Algorithmic bytes of one global iteration (one pull over the whole CSR):
    col_idx 4 B per entry, row pointers 4 B per node, and per node x, r, h
    read-modify-write plus one write and one read of its scatter value z."""
    return 4 * nnz + 4 * (n + 1) + 8 * vsize * n


def sub_global_roofline(ctx, g, G, seeds, dev):
    """Global GD (every node, every iteration) on the benchmark graph in FP32 at
    eps 1e-7 from four of the batch's seeds: time per iteration of the pull
    kernel and its achieved algorithmic bandwidth."""
    import torch

    from paper_2410_21634_amd import gde

    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float32, device=dev)
    p = gde.make_params("ppr", "gd", alpha=0.1, eps=1e-7, value_type=gde.F32)
    gde.solve_global(ctx, g, p, [int(seeds[0])], out=(oi, ov))
    torch.cuda.synchronize()
    ctx.profile(True, reset=True)
    iters = 0
    t = time.perf_counter()
    for s in seeds[::256][:4]:
        r = gde.solve_global(ctx, g, p, [int(s)], out=(oi, ov))
        iters += r.iters
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    prof = ctx.profile(False, reset=True)
    it_ms = prof["total_ms"] / max(iters, 1)
    bpi = glob_bytes_per_iter(G.n, G.nnz, 4)
    ach = bpi / (it_ms * 1e-3) / 1e9 if it_ms > 0 else 0.0
    return dict(kernel="k_glob_step<float> (one pull over the whole CSR per iteration)", solves=4, iters=iters,
                us_per_iter=round(it_ms * 1e3, 2), alg_bytes_per_iter=bpi, achieved_gbs=round(ach, 1),
                frac=round(ach / PEAK_HBM_GBS, 4), ms_per_solve=round(1e3 * wall / 4, 3),
                timing="HIP events around each chunk of iteration launches (no-op launches after the stop "
                       "included), divided by the iterations that ran",
                byte_rule="4 B per CSR entry + 4 B per row pointer + 32 B per node (x, r, h read and written, "
                          "z written and read)")


def sub_global_vs_local(budget_s=90.0):
    """Local vs global solvers (the Table 2 and eps-sweep comparisons of Sec. 5)
    on the n = 10^6 power-law graph and the 1000 x 1000 grid, PPR alpha 0.1, FP64,
    8 uniform sources per graph: operations (sum vol(S_t) vs T * nnz) and median
    wall time per solve for LocalGD vs GD over eps = 2^-17 ... 2^-32, and the
    operation ratios GD/LocalGD and CH/LocalCH at eps = 1/n."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    dev = torch.device("cuda:0")
    out = dict(workload="PPR alpha 0.1, FP64, 8 uniform sources per graph; graphs: Chung-Lu n=1e6, 1e7 edges, "
                        "gamma 2.5, seed 42, and the 1000x1000 4-neighbour grid (1,998,000 edges)",
               eps_sweep=[2.0 ** -k for k in (17, 20, 23, 26, 29, 32)])
    t_all = time.perf_counter()
    for gname, G in (("chung_lu_n1M", W.chung_lu(1_000_000, 10_000_000, 2.5, seed=42)),
                     ("grid_1000x1000", W.grid_2d(1000, 1000))):
        ctx = gde.Context(0)
        rp = torch.from_numpy(G.row_ptr).to(dev)
        ci = torch.from_numpy(G.col_idx).to(dev)
        g = gde.Graph(ctx, rp, ci)
        seeds = [int(s) for s in W.uniform_seeds(G, 8, seed=42)]
        oi = torch.empty(G.n, dtype=torch.int32, device=dev)
        ov = torch.empty(G.n, dtype=torch.float64, device=dev)

        def timed(fn, p):
            ts, ops = [], []
            for s in seeds:
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = fn(ctx, g, p, [s], out=(oi, ov))
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
                ops.append(r.ops)
            return float(np.median(ts)) * 1e3, float(np.mean(ops))

        rec = dict(n=G.n, nnz=G.nnz, sweep=[])
        # Table 2 analogue at eps = 1/n: operation ratios of the standard solvers over the local ones
        e_n = 1.0 / G.n
        ratios = {}
        for m in ("gd", "ch"):
            p = gde.make_params("ppr", m, alpha=0.1, eps=e_n, value_type=gde.F64, max_iters=100000)
            _, lo = timed(gde.solve, p)
            _, go = timed(gde.solve_global, p)
            ratios[m] = round(go / lo, 2)
        rec["ops_ratio_at_eps_1_over_n"] = dict(gd_over_localgd=ratios["gd"], ch_over_localch=ratios["ch"])
        for e in out["eps_sweep"]:
            if time.perf_counter() - t_all > budget_s:
                rec["sweep"].append(dict(eps=e, skipped="time budget"))
                continue
            p = gde.make_params("ppr", "gd", alpha=0.1, eps=e, value_type=gde.F64, max_iters=100000)
            gde.solve(ctx, g, p, [seeds[0]], out=(oi, ov))
            l_ms, l_ops = timed(gde.solve, p)
            g_ms, g_ops = timed(gde.solve_global, p)
            rec["sweep"].append(dict(eps=e, local_ms=round(l_ms, 3), global_ms=round(g_ms, 3),
                                     local_ops=round(l_ops), global_ops=round(g_ops),
                                     time_speedup=round(g_ms / l_ms, 2), ops_ratio=round(g_ops / l_ops, 2)))
            log(f"global vs local {gname} eps 2^{np.log2(e):.0f}: local {l_ms:.3f} ms, global {g_ms:.3f} ms")
        faster = [r["eps"] for r in rec["sweep"] if "local_ms" in r and r["local_ms"] <= r["global_ms"]]
        rec["smallest_eps_local_faster"] = min(faster) if faster else None
        out[gname] = rec
        g.close()
        ctx.close()
        del rp, ci
        torch.cuda.empty_cache()
    return out


def sub_sor(n_seeds=256):
    """LocalSOR at omega* and APPR (the FIFO push, one query per wavefront)
    against batched LocalGD as eps shrinks, on an ogbn-arxiv-sized Chung-Lu
    graph (n = 169,343, 1,166,243 edges), PPR alpha 0.1: the comparison of
    Fig. 5.  Solves/s of one gde_solve_batch call per method and eps, and the
    mean operations (sum of d_u over the pushes) of its queries."""
    import math

    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    G = W.chung_lu(169_343, 1_166_243, 2.5, seed=42)
    seeds = [int(s) for s in W.uniform_seeds(G, n_seeds, seed=42)]
    ctx = gde.Context(0)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    om_star = 2.0 / (1.0 + math.sqrt(1.0 - 0.9 ** 2))
    cap = G.n
    bo = (torch.empty(n_seeds * cap, dtype=torch.int32, device=dev),
          torch.empty(n_seeds * cap, dtype=torch.float32, device=dev))
    methods = (("localgd", "gd", 0.0), ("appr", "sor", 1.0), ("localsor_omega_star", "sor", om_star))
    out = dict(workload=f"Chung-Lu n=169,343, 1,166,243 edges, gamma 2.5, seed 42; {n_seeds} uniform seeds; "
                        "PPR alpha 0.1; one gde_solve_batch call per method and eps (FP32 output; LocalSOR and "
                        "APPR keep FP64 state)",
               omega_star=round(om_star, 4), nnz=int(len(G.col_idx)), per_eps={})
    for i, eps in enumerate((1e-6, 1e-7, 1e-8)):
        rec = {}
        for name, method, om in methods:
            ps = [gde.make_params("ppr", method, alpha=0.1, eps=eps, omega=om, value_type=gde.F32) for _ in seeds]
            if i == 0:  # first call per method sizes the workspaces
                gde.solve_batch(ctx, g, ps, [([s], None) for s in seeds], out=bo)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = gde.solve_batch(ctx, g, ps, [([s], None) for s in seeds], out=bo)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            assert (np.asarray(res.status) == gde.OK).all(), name
            rec[name] = dict(solves_per_s=round(n_seeds / dt, 1), mean_ops=round(float(res.ops.mean()), 1),
                             mean_pushes=round(float(res.pushes.mean()), 1))
        rec["mean_ops_over_nnz_appr"] = round(rec["appr"]["mean_ops"] / len(G.col_idx), 3)
        rec["ops_sor_star_over_appr"] = round(rec["localsor_omega_star"]["mean_ops"] / rec["appr"]["mean_ops"], 3)
        out["per_eps"][f"{eps:g}"] = rec
        log(f"sor eps {eps:g}: " + ", ".join(f"{k} {v['solves_per_s']}/s ops {v['mean_ops']:.3g}"
                                             for k, v in rec.items() if isinstance(v, dict)))
    g.close()
    ctx.close()
    del rp, ci, bo
    torch.cuda.empty_cache()
    return out


def sub_dynamic():
    """Standing queries under graph snapshots (the analogue of the paper's dynamic
    PPR experiment, Sec. 5): an ogbn-arxiv-sized Chung-Lu graph (n = 169,343,
    1,166,243 edges, gamma 2.5), 17.9 % of its edges at the start and the rest
    in 16 insertion batches (and a variant where every batch also deletes 10 % of
    its size), 16 PPR queries (alpha 0.1, eps = 1e-2 / n, FP64).  Accumulated
    operations (sum vol(S_t)) and time of the dynamic path (corrections and warm
    re-solve, gde_dyn_update) against solving every query from scratch on each
    snapshot (gde_solve)."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    G = W.chung_lu(169_343, 1_166_243, 2.5, seed=42)
    n = G.n
    eps = 1e-2 / n
    out = dict(workload="Chung-Lu n=169,343, 1,166,243 edges, gamma 2.5, seed 42; 17.9% of the edges at start, "
                        "16 batches; 16 uniform sources of graph 0 (deletions spare their edges); PPR alpha 0.1, eps 1e-2/n, FP64")
    dev = torch.device("cuda:0")
    for name, dfrac in (("insert", 0.0), ("insert_delete", 0.1)):
        g0, _ = W.snapshots(G, 16, 0.179, 0.0, seed=42)
        seeds = [int(s) for s in W.uniform_seeds(g0, 16, seed=42)]
        g0, batches = W.snapshots(G, 16, 0.179, dfrac, seed=42, protect=seeds)
        ctx = gde.Context(0)
        rp = torch.from_numpy(g0.row_ptr).to(dev)
        ci = torch.from_numpy(g0.col_idx).to(dev)
        g = gde.Graph(ctx, rp, ci)
        p = gde.make_params("ppr", alpha=0.1, eps=eps, value_type=gde.F64)
        dyn = gde.Dynamic(ctx, g, value_type=gde.F64)
        qids = [dyn.add(p, [s]) for s in seeds]
        ops0 = sum(dyn.read(q).ops for q in qids)
        dyn_ops, st_ops, dyn_ms, st_ms = [ops0], [ops0], [], []
        oi = torch.empty(n, dtype=torch.int32, device=dev)
        ov = torch.empty(n, dtype=torch.float64, device=dev)
        for iu, iv, du, dv in batches:
            t = time.perf_counter()
            dyn.update(insert=np.stack([iu, iv], axis=1), delete=np.stack([du, dv], axis=1))
            dyn_ms.append(1e3 * (time.perf_counter() - t))
            dyn_ops.append(dyn_ops[-1] + sum(dyn.read(q).ops for q in qids))
            gv = dyn.graph
            gde.solve(ctx, gv, p, [seeds[0]], out=(oi, ov))  # the new version's workspace, untimed
            torch.cuda.synchronize()
            t = time.perf_counter()
            ops = 0
            for s in seeds:
                ops += gde.solve(ctx, gv, p, [s], out=(oi, ov)).ops
            torch.cuda.synchronize()
            st_ms.append(1e3 * (time.perf_counter() - t))
            st_ops.append(st_ops[-1] + ops)
        log(f"dynamic {name}: accumulated ops dynamic {dyn_ops[-1]} static {st_ops[-1]}")
        out[name] = dict(accumulated_ops_dynamic=dyn_ops, accumulated_ops_static=st_ops,
                         ops_ratio_static_over_dynamic=round(st_ops[-1] / max(dyn_ops[-1], 1), 2),
                         ms_per_batch_dynamic=round(float(np.mean(dyn_ms)), 3),
                         ms_per_batch_static=round(float(np.mean(st_ms)), 3),
                         timing="dynamic: gde_dyn_update (host event checks, CSR rebuild and upload, corrections "
                                "and one batched warm re-solve of all 16 queries); static: 16 gde_solve calls")
        dyn.close()
        g.close()
        ctx.close()
        del rp, ci
        torch.cuda.empty_cache()
    return out


def serve_sweep(args, ctx, g, G, qps_list, warm_s, serve_s):
    """Open-loop Poisson arrivals of mixed PPR / Katz / HK queries (kind uniform,
    half single seeds, half 8-node seed sets, eps log-uniform [1e-7, 1e-4] for
    every kind) with a 10,000-edge insert batch every 100 ms, at each rate of
    qps_list.  Queries and insert batches are drawn before the clock starts;
    latency is harvest time minus scheduled arrival time."""
    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    lo, hi = g.lambda_max(max_iters=300, rtol=1e-3)
    beta = 0.5 / hi
    log(f"lambda bounds [{lo:.3f}, {hi:.3f}], beta {beta:.4g}")
    total_s = warm_s + serve_s
    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    existing = set()
    inserts = [W.insert_batch(G, args.insert_k, rng, existing) for _ in range(int(total_s / 0.1))]
    log(f"{len(inserts)} insert batches of {args.insert_k} drawn in {time.perf_counter() - t0:.1f}s")
    pool = W.stratified_seeds(G, 4096, bins=16, seed=7)
    sets = [W.seed_set(G, int(a), 8, rng) for a in pool[::4]]
    results = []
    for qps in qps_list:
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
                p = gde.make_params("katz", beta=beta, eps=e, lambda_bound=hi)
            else:
                p = gde.make_params("hk", tau=5.0, K=30, eps=e)
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
                submitted += arr[i] >= warm_s
                kinds[qs[i][3]][1] += int(arr[i] >= warm_s)
                i += 1
            while ins < len(inserts) and (ins + 1) * 0.1 <= now:
                srv.insert_edges(*inserts[ins])
                ins += 1
            done = srv.poll()
            tn = time.perf_counter() - t0
            for c in done:
                t_arr = sub_at.pop(c["ticket"])
                kd = kinds[sub_kind.pop(c["ticket"])]
                if t_arr >= warm_s:
                    lat.append(tn - t_arr)
                    completed += 1
                    kd[0] += 1
                    kd[2].append((tn - t_arr) * 1e3)
            if i >= len(arr) and not sub_at:
                break
        srv.close()
        lat_ms = np.array(lat) * 1e3
        offered = int(np.sum(arr >= warm_s))
        rec = dict(qps=qps, submitted=int(submitted), completed=int(completed), offered=offered,
                   completion_ratio=round(completed / max(offered, 1), 4),
                   solves_per_s=round(completed / serve_s, 2), inserted_edges=ins * args.insert_k,
                   p50_ms=round(float(np.percentile(lat_ms, 50)), 3) if len(lat_ms) else None,
                   p99_ms=round(float(np.percentile(lat_ms, 99)), 3) if len(lat_ms) else None,
                   by_kind={k: dict(completed=int(v[0]), submitted=int(v[1]),
                                    p50_ms=round(float(np.percentile(v[2], 50)), 3) if v[2] else None,
                                    p99_ms=round(float(np.percentile(v[2], 99)), 3) if v[2] else None)
                            for k, v in kinds.items()})
        log(f"serve {rec}")
        results.append(rec)
    ok = [r for r in results if r["completion_ratio"] >= 0.99]
    stated = max(ok, key=lambda r: r["qps"]) if ok else None
    return stated, results


def run_serve_sub(args, ctx, g, G):
    """A short serving sweep on the n = 10^7 graph already on the device: each
    rate of --serve-sub-qps for 1 s of warm-up and --serve-sub-s seconds measured."""
    stated, results = serve_sweep(args, ctx, g, G, args.serve_sub_qps, 1.0, args.serve_sub_s)
    return dict(workload=f"serving: the n=1e7 graph; Poisson arrivals of mixed PPR/Katz/HK (kind uniform, half single "
                         f"seeds, half 8-node seed sets, eps log-uniform [1e-7,1e-4]), {args.insert_k}-edge inserts "
                         f"every 100 ms; 1 s warm-up + {args.serve_sub_s:g} s measured per rate",
                stated_qps=stated["qps"] if stated else None,
                stated_rule="highest swept rate with >= 99% of the offered queries completed",
                latency_ms=dict(p50=stated["p50_ms"], p99=stated["p99_ms"]) if stated else None, sweep=results)


def run_serve(args):
    """Serving sweep as its own JSON line (--workload serve)."""
    import torch

    from paper_2410_21634_amd import gde
    from paper_2410_21634_amd import workloads as W

    ctx = gde.Context(0)
    n, E = (10_000_000, 200_000_000) if not args.small else (1_000_000, 10_000_000)
    t0 = time.perf_counter()
    G = W.chung_lu(n, E, 2.2, seed=42)
    log(f"graph {G.summary()} built in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    stated, results = serve_sweep(args, ctx, g, G, args.qps, args.warm_s, args.serve_s)
    head = stated or results[0]
    out = dict(metric=METRIC, value=head["solves_per_s"], unit="solves/s", n_gpus=1, steps=len(results),
               warmup=0, ms_per_step=None, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=f"serving: Chung-Lu n={n}, {E} edges, gamma 2.2; Poisson arrivals of mixed "
                                    f"PPR/Katz/HK (eps log-uniform [1e-7,1e-4] for every kind), {args.insert_k}-edge "
                                    f"inserts every 100 ms",
                           stated_qps=stated["qps"] if stated else None, serve_s=args.serve_s, warm_s=args.warm_s),
               latency_ms=dict(p50=head["p50_ms"], p99=head["p99_ms"]), sweep=results)
    g.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=["c2", "c4", "serve", "global", "dynamic", "sor"],
                    help="global / dynamic / sor: only the local-vs-global, snapshot or LocalSOR record")
    ap.add_argument("--plain-sample", type=int, default=1024,
                    help="c4: plain solves timed for the comparison (1,024 = every query of the batch)")
    ap.add_argument("--no-sub", action="store_true", help="c4: skip the serving and other-config sub-records")
    ap.add_argument("--serve-sub-qps", type=float, nargs="+", default=[2000, 5000, 10000])
    ap.add_argument("--serve-sub-s", type=float, default=4.0)
    ap.add_argument("--qps", type=float, nargs="+", default=[1000, 2000, 5000, 10000, 20000, 50000])
    ap.add_argument("--warm-s", type=float, default=2.0)
    ap.add_argument("--serve-s", type=float, default=10.0)
    ap.add_argument("--insert-k", type=int, default=10000)
    ap.add_argument("--groups", type=int, default=16)
    ap.add_argument("--iters-per-step", type=int, default=4)
    ap.add_argument("--small", action="store_true", help="serve: the n=1e6 graph instead of n=1e7")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--phase", default="all", choices=["all", "plain", "batch"],
                    help="profiling aid: run only one path (the JSON line then covers that path only)")
    ap.add_argument("--schedule", default='{"auto":1}',
                    help='batched schedule JSON, e.g. {"lanes":16}; default: chosen by the library\'s autotuner')
    ap.add_argument("--pmc-summary", nargs=3, metavar=("TARGET", "FETCH_DIR", "WRITE_DIR"),
                    help="TARGET plain|batch: write profiles/<target summary>.json, the per-launch traffic from "
                         "two rocprofv3 --pmc runs, and exit")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time the scatter launches of every k-th plain solve with HIP events")
    ap.add_argument("--copy-calib", action="store_true",
                    help="end with one elementwise multiply over 2 GiB (2 GiB read, 2 GiB written), the calibration "
                         "for the HBM byte counters")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print(json.dumps(dict(error="bench.py measures one GPU only; multi-GPU sharding is by query "
                                    "(replicated graph) and is described, not run")), flush=True)
        sys.exit(2)
    if args.workload == "global":
        out = sub_global_vs_local(budget_s=1e9)
    elif args.workload == "dynamic":
        out = sub_dynamic()
    elif args.workload == "sor":
        out = sub_sor()
    else:
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
