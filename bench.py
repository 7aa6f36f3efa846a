#!/usr/bin/env python3
"""Benchmark of the s-line-graph build on one MI355X.

Default workload: the power-law hypergraph with 1,000,000 hyperedges over
2,000,000 vertices (sizes truncated Zipf 2.2 on [2, 1e4], vertex popularity
truncated Zipf 1.8 on [1, 1e5], seed 21), int32 CSR resident in HBM.  One step
builds L_s(H) for every s in {1, 2, 4, 8, 16} with one plain sline_build call
each (outputs stay on the device; they are freed before the next call).

Printed: one JSON line with incidence entries/s over the whole step, the
roofline of the dominant kernel (the workgroup counting kernel k_count_tasks:
algorithmic bytes 12*nnz + 4*W + 8*P of the items it counts -- their
incidences, wedges and the (b, w) pairs it stages -- over its run time, HIP
events on the library's stream around that kernel alone) and the CPU oracle
timed on a bounded sample of the same workload.  HBM traffic comes from the
committed rocprofv3 counter summary of that kernel when the kernel source is
unchanged since it was taken (else null).

Other forms (--form): ``dual`` (the same graph's dual, s in {2, 8, 32});
``batch`` (512 graphs of the batched-workload law, each with its own s: one
sline_build_batch call per step against one sline_build call per graph, same
graphs, same GPU; --autotune first tunes the launch parameters on the batch);
``serve`` (a catalog of batch-law graphs plus power-law graphs of the
1,000,000 x 2,000,000 size, queried by Poisson arrivals at 200/s with s on
1..16 and a random side through the serving loop: p50/p99 latency from
submit to result on the device, throughput, and the same queries run back to
back with one plain call each); ``copy`` (a plain device copy of known size,
the calibration run for the FETCH_SIZE / WRITE_SIZE counters).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(ROOT, "paper_2010_11448_amd", "csrc", "sline_count.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_count_tasks_powerlaw_1Mx2M_traffic.md")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--form", default="plain", choices=["plain", "dual", "batch", "serve", "copy"])
    p.add_argument("--duration", type=float, default=20.0, help="serve form: seconds of arrivals")
    p.add_argument("--rate", type=float, default=200.0, help="serve form: arrivals per second")
    p.add_argument("--catalog-small", type=int, default=256)
    p.add_argument("--catalog-large", type=int, default=2)
    p.add_argument("--budget-gb", type=float, default=160.0)
    p.add_argument("--workers", type=int, default=3)
    p.add_argument("--graphs", type=int, default=512, help="batch form: number of graphs")
    p.add_argument("--spgemm", action="store_true",
                   help="plain/dual forms: take the product route (sline_build_spgemm)")
    p.add_argument("--autotune", action="store_true", help="batch form: tune launch parameters first")
    p.add_argument("--tune-budget", type=float, default=90.0)
    p.add_argument("--s", default=None, help="comma-separated s values")
    p.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=0, help="rows in the CPU sample (0 = auto)")
    return p.parse_args()


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else None


def cpu_baseline(g, s_list, dual, rows_hint, budget_s=20.0):
    """The O1 oracle (all pairs, sorted merge) on a seeded sample of items.

    Rows a are drawn uniformly; the oracle compares each with every b > a,
    so the sampled time scaled by N / rows estimates the full build.  The
    sample size is set from a short probe aimed at `budget_s` seconds for the
    whole sweep; the probe overstates the cost per row somewhat (threads wait
    for their slowest rows), so the sweep takes about 10-20 s."""
    import oracle

    N = g.n_vertices if dual else g.n_edges
    threads = min(os.cpu_count() or 1, 16)
    rng = np.random.default_rng(12345)
    order = rng.permutation(N).astype(np.int32)
    if rows_hint:
        nrows = rows_hint
    else:
        # several rows per thread, so the probe's wall time is not set by
        # the one slowest row of a thread
        probe = np.sort(order[:threads * 8])
        t0 = time.perf_counter()
        oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s_list[0], dual=dual, rows=probe,
                     threads=threads, keep=False)
        per_row = max((time.perf_counter() - t0) / len(probe), 1e-6)
        nrows = int(budget_s / (per_row * len(s_list)))
    nrows = max(threads, min(nrows, N))
    rows = np.sort(order[:nrows])
    est = 0.0
    spent = 0.0
    for s in s_list:
        t0 = time.perf_counter()
        oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, rows=rows,
                     threads=threads, keep=False)
        dt = time.perf_counter() - t0
        spent += dt
        est += dt * N / len(rows)
    value = len(s_list) * g.nnz / est
    return {"value": value, "unit": "incidence entries/s", "cores": threads, "kind": "oracle",
            "sample": f"O1 naive all-pairs oracle on {len(rows)} uniformly drawn items of {N} "
                      f"(every b > a compared), s in {list(s_list)}; {spent:.1f} s measured, "
                      f"scaled by N/rows to {est:.0f} s for the full sweep"}


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_traffic(form):
    """HBM bytes per launch of the task kernel from the committed counter
    summary, if it was taken on the current kernel source and this form."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"^traffic_json: (\{.*\})$", text, re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_sha") != kernel_sha() or rec.get("form") != form:
        return None
    return rec


def copy_calibration(steps):
    """A plain device copy of known size, for calibrating HBM counters."""
    import torch

    nbytes = 1 << 31
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    print(json.dumps({"form": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "ms": dt * 1e3, "GBps": 2 * nbytes / dt / 1e9}), flush=True)


def bench_batch(args, ctx, dev):
    """Batched form: one sline_build_batch call vs one sline_build call per graph."""
    import torch

    from paper_2010_11448_amd import autotune, gen, sline

    print(f"bench: generating {args.graphs} batch graphs", file=sys.stderr, flush=True)
    items = gen.batch_workload(args.graphs)
    graphs = [(torch.from_numpy(it.graph.row_ptr).to(dev), torch.from_numpy(it.graph.col).to(dev),
               it.graph.n_vertices) for it in items]
    s_list = [it.s for it in items]
    dual = [it.dual for it in items]
    nnz = sum(it.graph.nnz for it in items)
    flags = sline.SLINE_PROFILE

    # both sides let the library allocate the results (one call per build)
    def run_batch():
        outs = ctx.build_batch_owned(graphs, s_list, dual, flags)
        ctx.free_edges(outs, len(graphs))

    def run_plain():
        for (rp, col, nv), s, d in zip(graphs, s_list, dual):
            out = ctx.build_owned(rp, col, nv, s, d, flags)
            ctx.free_edges([out])

    tuned = None
    if args.autotune:
        print("bench: autotuning on the batch", file=sys.stderr, flush=True)
        tuned, _ = autotune.tune(ctx, run_batch, budget_s=args.tune_budget,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
    for _ in range(max(args.warmup, 1)):
        run_batch()
        run_plain()
    torch.cuda.synchronize()
    tb = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        run_batch()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        print(f"bench: batch step {i + 1}/{args.steps} {tb[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    st = ctx.stats()
    tp = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        run_plain()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
        print(f"bench: plain step {i + 1}/{args.steps} {tp[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    t_batch = sum(tb) / len(tb)
    t_plain = sum(tp) / len(tp)
    b = 12.0 * st["heavy_nnz"] + 4.0 * st["heavy_wedges"] + 8.0 * st["heavy_pairs"]
    ach = b / 1e9 / (st["ms_tasks"] / 1e3) if st["ms_tasks"] > 0 else 0.0
    line = {
        "metric": "s-line graph build: incidence entries/s, % HBM peak; batched vs plain; p50/p99",
        "value": nnz / t_batch, "unit": "incidence entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batch_lognormal_{args.graphs}", "graphs": args.graphs, "nnz": nnz,
                   "items": sum(it.graph.n_edges for it in items), "s": "per graph, uniform on 1..12"},
        "batch": {"batched_entries_per_s": nnz / t_batch, "plain_entries_per_s": nnz / t_plain,
                  "batched_vs_plain": t_plain / t_batch, "batched_p50_ms": pct([x * 1e3 for x in tb], 50),
                  "batched_p99_ms": pct([x * 1e3 for x in tb], 99),
                  "plain_p50_ms": pct([x * 1e3 for x in tp], 50),
                  "plain_p99_ms": pct([x * 1e3 for x in tp], 99),
                  "pairs": st["n_pairs"], "tuning": tuned or ctx.tuning(),
                  "batched_stage_ms": {k: st[k] for k in ("ms_transpose", "ms_prepare", "ms_count",
                                                          "ms_scan", "ms_fill", "ms_tasks")}},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_count_tasks (one launch per batched build)",
                     "alg_bytes_per_launch": "12*nnz + 4*W + 8*P over the items it counts",
                     "alg_bytes_mean": b, "ms_mean": st["ms_tasks"]},
    }
    print(json.dumps(line), flush=True)


def bench_serve(args, dev):
    """Serving form: Poisson arrivals through the query loop, then the same
    queries with one plain call each."""
    import torch

    from paper_2010_11448_amd import gen, sline

    print("bench: generating the serving catalog", file=sys.stderr, flush=True)
    cat = [gen.batch_graph(g).graph for g in range(args.catalog_small)]
    cat += [gen.powerlaw_1m(seed=21 + i) for i in range(args.catalog_large)]
    dgr = [(torch.from_numpy(h.row_ptr).to(dev), torch.from_numpy(h.col).to(dev), h.n_vertices)
           for h in cat]
    qs = gen.serving_arrivals(args.catalog_small, args.catalog_large, rate=args.rate,
                              duration_s=args.duration)
    srv = sline.Server(0, hbm_budget_bytes=int(args.budget_gb * (1 << 30)), max_batch=64,
                       workers=args.workers)
    ids = [srv.register(rp, col, n) for rp, col, n in dgr]
    # warm the server: a few queries, and the largest result of each large
    # graph (maps the device memory its cache will reuse)
    warm = [(ids[q.graph_id], q.s, q.dual) for q in qs[:8]]
    warm += [(ids[args.catalog_small + i], 1, 0) for i in range(args.catalog_large)]
    for gid, s_, d_ in warm:
        t = srv.submit(gid, s_, d_)
        while srv.poll(t, keep=False) is None:
            time.sleep(0.0005)
    print(f"bench: serving {len(qs)} queries over {args.duration:.0f} s", file=sys.stderr, flush=True)
    infos = {}
    outstanding = []
    t0 = time.perf_counter()
    k = 0
    last_print = t0
    while k < len(qs) or outstanding:
        now = time.perf_counter() - t0
        while k < len(qs) and qs[k].arrival_s <= now:
            q = qs[k]
            outstanding.append((srv.submit(ids[q.graph_id], q.s, q.dual), k))
            k += 1
        still = []
        for t, i in outstanding:
            r = srv.poll(t, keep=False)
            if r is None:
                still.append((t, i))
            else:
                infos[i] = r[1]
        outstanding = still
        if time.perf_counter() - last_print > 5.0:
            last_print = time.perf_counter()
            qd, rn = srv.pending()
            print(f"bench: served {len(infos)}/{len(qs)} (submitted {k}, queued {qd}, "
                  f"running batches {rn})", file=sys.stderr, flush=True)
        if k < len(qs):
            time.sleep(max(0.0, min(0.0005, qs[k].arrival_s - (time.perf_counter() - t0))))
        else:
            time.sleep(0.0002)
    wall = time.perf_counter() - t0
    lat = [(infos[i]["t_done_ns"] - infos[i]["t_submit_ns"]) / 1e6 for i in range(len(qs))]
    nnz = sum(cat[q.graph_id].nnz for q in qs)
    batch_sizes = [infos[i]["batch_size"] for i in range(len(qs))]
    first = min(infos[i]["t_submit_ns"] for i in range(len(qs)))
    last = max(infos[i]["t_done_ns"] for i in range(len(qs)))
    # saturation: every query submitted at once; results are taken (and
    # released) as they complete, in any order
    t1 = time.perf_counter()
    ts = [srv.submit(ids[q.graph_id], q.s, q.dual) for q in qs]
    while ts:
        ts = [t for t in ts if srv.poll(t, keep=False) is None]
        if ts:
            time.sleep(0.0002)
    t_sat = time.perf_counter() - t1
    srv.close()
    print("bench: plain calls, one per query", file=sys.stderr, flush=True)
    ctx = sline.Context(0)
    t2 = time.perf_counter()
    t_plain_large = 0.0
    for q in qs:
        rp, col, n = dgr[q.graph_id]
        tq = time.perf_counter()
        out = ctx.build_owned(rp, col, n, q.s, q.dual)
        ctx.free_edges([out])
        if q.graph_id >= args.catalog_small:
            torch.cuda.synchronize()
            t_plain_large += time.perf_counter() - tq
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t2
    ctx.close()
    large = [lat[i] for i, q in enumerate(qs) if q.graph_id >= args.catalog_small]
    line = {
        "metric": "s-line graph build: incidence entries/s, % HBM peak; batched vs plain; p50/p99",
        "value": nnz / t_sat, "unit": "incidence entries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_sat * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"serving_poisson{args.rate:.0f}_{args.duration:.0f}s",
                   "queries": len(qs), "catalog_small": args.catalog_small,
                   "catalog_large": args.catalog_large, "budget_gb": args.budget_gb,
                   "workers": args.workers},
        "serve": {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": max(lat),
                  "large_p50_ms": pct(large, 50), "large_p99_ms": pct(large, 99),
                  "queries_per_s_arrival_run": len(qs) / ((last - first) / 1e9),
                  "entries_per_s_arrival_run": nnz / ((last - first) / 1e9),
                  "wall_s": wall, "mean_batch": sum(batch_sizes) / len(batch_sizes),
                  "max_batch": max(batch_sizes),
                  "saturation_s": t_sat, "saturation_queries_per_s": len(qs) / t_sat,
                  "plain_s": t_plain, "plain_large_s": t_plain_large,
                  "plain_queries_per_s": len(qs) / t_plain,
                  "served_vs_plain": t_plain / t_sat},
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rows of the result shard across GPUs without exchange)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2010_11448_amd import gen, sline

    if args.form == "copy":
        copy_calibration(max(args.steps, 1))
        return
    dev = torch.device("cuda", 0)
    if args.form == "batch":
        ctx = sline.Context(0)
        bench_batch(args, ctx, dev)
        ctx.close()
        return
    if args.form == "serve":
        bench_serve(args, dev)
        return
    dual = 1 if args.form == "dual" else 0
    s_list = tuple(int(x) for x in args.s.split(",")) if args.s else (
        gen.DUAL_S if dual else gen.POWERLAW_S)
    print(f"bench: generating workload (scale {args.scale})", file=sys.stderr, flush=True)
    g = gen.powerlaw_1m(scale=args.scale)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    ctx = sline.Context(0)
    flags = sline.SLINE_PROFILE
    per_s = {s: [] for s in s_list}

    def step(record):
        for s in s_list:
            t0 = time.perf_counter()
            L = ctx.build(rp, col, g.n_vertices, s, dual, flags, spgemm=args.spgemm)
            t1 = time.perf_counter()
            if record:
                per_s[s].append((t1 - t0, ctx.stats()))
            del L

    for i in range(args.warmup):
        step(False)
        print(f"bench: warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        print(f"bench: step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / max(args.steps, 1)
    value = len(s_list) * g.nnz / (ms_per_step / 1000.0)

    alg_bytes = 0.0
    task_ms = 0.0
    launches = 0
    builds = {}
    for s in s_list:
        recs = per_s[s]
        times = [r[0] * 1000.0 for r in recs]
        st = recs[0][1]
        b = 12.0 * st["heavy_nnz"] + 4.0 * st["heavy_wedges"] + 8.0 * st["heavy_pairs"]
        for _, sr in recs:
            alg_bytes += b
            task_ms += sr["ms_tasks"]
            launches += 1
        builds[str(s)] = {
            "p50_ms": pct(times, 50), "p99_ms": pct(times, 99),
            "pairs": st["n_pairs"], "wedges": st["wedges"], "kept_items": st["n_kept"],
            "task_kernel_alg_bytes": b, "ms_tasks": float(np.median([r[1]["ms_tasks"] for r in recs])),
            "task_kernel_GBps": b / 1e6 / max(float(np.median([r[1]["ms_tasks"] for r in recs])), 1e-9),
            "ms_transpose": float(np.median([r[1]["ms_transpose"] for r in recs])),
            "ms_prepare": float(np.median([r[1]["ms_prepare"] for r in recs])),
            "ms_count": float(np.median([r[1]["ms_count"] for r in recs])),
            "ms_scan": float(np.median([r[1]["ms_scan"] for r in recs])),
            "ms_fill": float(np.median([r[1]["ms_fill"] for r in recs])),
            "heavy_items": st["n_heavy"], "small_items": st["n_small"], "passes": st["passes"],
            "product_nnz": st["product_nnz"], "ms_product": st["ms_product"],
            "ms_filter": st["ms_filter"],
        }
    achieved = alg_bytes / 1e9 / (task_ms / 1000.0) if task_ms > 0 else 0.0
    tr = committed_traffic(args.form if args.scale == 1.0 and not args.s else None)
    traffic = tr["bytes_per_launch"] if tr else None
    line = {
        "metric": "s-line graph build: incidence entries/s, % HBM peak; batched vs plain; p50/p99",
        "value": value,
        "unit": "incidence entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": g.meta.get("workload", "powerlaw") + (" dual" if dual else "") +
                   (" spgemm" if args.spgemm else ""),
                   "n_edges": g.n_edges, "n_vertices": g.n_vertices, "nnz": g.nnz,
                   "s": list(s_list), "dual": dual, "builds_per_step": len(s_list)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_count_tasks (workgroup counting kernel, one launch per build)",
                     "alg_bytes_per_launch": "12*nnz + 4*W + 8*P over the items it counts",
                     "alg_bytes_mean": alg_bytes / max(launches, 1),
                     "ms_mean": task_ms / max(launches, 1), "launches": launches,
                     "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT) if tr else None},
        "builds": builds,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, s_list, dual, args.cpu_rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
