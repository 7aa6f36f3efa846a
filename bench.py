#!/usr/bin/env python3
"""Benchmark of the s-line-graph build on one MI355X.

Default workload (the timed ``value``): the power-law hypergraph with
1,000,000 hyperedges over 2,000,000 vertices (sizes truncated Zipf 2.2 on
[2, 1e4], vertex popularity truncated Zipf 1.8 on [1, 1e5], seed 21), int32
CSR resident in HBM.  One step builds L_s(H) for every s in {1, 2, 4, 8, 16}
with one plain sline_build call each (outputs stay on the device; they are
freed before the next call).

The one JSON line carries, beside ``value``:

* ``roofline`` -- the dominant kernel (the workgroup counting kernel
  k_count_tasks): algorithmic bytes 12*nnz + 4*W + 8*P of the items it counts
  (their incidences, wedges and the (b, w) pairs it stages) over its run time,
  HIP events on the library's stream around that kernel alone; HBM traffic
  from the committed rocprofv3 counter summary of that kernel when the kernel
  source is unchanged since it was taken (else null).  ``build_frac`` is the
  whole build's share of HBM peak under 12*nnz_s + 4*W_s + 12*|L_s|.
* ``cpu_baseline`` -- the wedge oracle O3 (the alternative algorithm of
  Sec. IV-B with exact counters), measured over every row of the same workload
  at s = 8 and 16 on the host's cores (16 threads, median of 3; one thread at
  s = 16 once), with the CPU model.
* ``uniform`` -- the 2,000 x 5,000 uniform workload, s = 1..8, three seeds.
* ``batch`` -- 512 graphs of the batched-workload law, each with its own s:
  one sline_build_batch call against one sline_build call per graph.
* ``serve`` -- a catalog of 1024 batch-law graphs plus 8 power-law graphs of
  the 1,000,000 x 2,000,000 size, queried by Poisson arrivals at 200/s (s on
  1..16, a random side, 5 % of queries on the large graphs) through the
  serving loop: p50/p99 latency from submit to result on the device,
  throughput at saturation, and the same queries run back to back with one
  plain call each.

* ``stages`` -- the rows after L_s: the s-sweep against plain builds,
  squeezing and components per s, relabel-by-degree both ways, and the
  variants f0..f4 of Table III at 1/20 scale with the oracle's heuristic
  algorithm timed beside them.

``--plain-only`` skips the last four.  Other forms (--form): ``dual`` (the
same graph's dual, s in {2, 8, 32}); ``batch`` and ``serve`` alone (with
--autotune, --duration and catalog options); ``copy`` (a plain device copy
of known size, the calibration run for the FETCH_SIZE / WRITE_SIZE
counters); ``cpu`` (the oracle over the whole sweep at 16 threads and at one
thread, median of 3, for the record).  --spgemm takes the product route.
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

HERE = os.path.dirname(os.path.abspath(__file__))
# autotuner cache shipped with the package (entries keyed by workload class)
TUNE_CACHE = os.path.join(HERE, "paper_2010_11448_amd", "tuning_cache.json")

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
# the counting kernels and their default launch parameters (Tuning): counter
# figures taken on other sources or defaults do not apply
KERNEL_SRCS = [os.path.join(ROOT, "paper_2010_11448_amd", "csrc", f)
               for f in ("sline_count.hip", "sline_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_count_tasks_powerlaw_1Mx2M_traffic.md")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--form", default="plain",
                   choices=["plain", "dual", "batch", "serve", "stages", "copy", "cpu"])
    p.add_argument("--plain-only", action="store_true",
                   help="plain form: skip the uniform, batch and serve sub-objects")
    p.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    p.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    p.add_argument("--catalog-small", type=int, default=1024)
    p.add_argument("--catalog-large", type=int, default=8)
    p.add_argument("--budget-gb", type=float, default=160.0)
    p.add_argument("--reuse-gb", type=float, default=REUSE_BYTES / (1 << 30),
                   help="serve: device memory for kept results (0: no result reuse)")
    p.add_argument("--workers", type=int, default=3)
    p.add_argument("--graphs", type=int, default=512, help="batch: number of graphs")
    p.add_argument("--batch-steps", type=int, default=5)
    p.add_argument("--spgemm", action="store_true",
                   help="plain/dual forms: take the product route (sline_build_spgemm)")
    p.add_argument("--autotune", action="store_true", help="batch form: tune launch parameters first")
    p.add_argument("--tune-budget", type=float, default=90.0)
    p.add_argument("--tune-cache", default=TUNE_CACHE,
                   help="batch form: autotuner cache; its entry for the batch's class is used "
                        "(with --autotune, the tuned setting is written to it)")
    p.add_argument("--s", default=None, help="comma-separated s values")
    p.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--gen-workers", type=int, default=16,
                   help="processes drawing the synthetic graphs (before the GPU is touched)")
    return p.parse_args()


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if xs else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    return max(1, min(os.cpu_count() or 1, 16))


def time_oracle(P, s, threads, reps):
    """Median wall time of O3 over every row of a prepared side."""
    import oracle

    ts = []
    st = None
    for _ in range(reps):
        t0 = time.perf_counter()
        _, st = oracle.wedge(None, None, 0, 0, s, threads=threads, keep=False, prepared=P)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), st


def cpu_baseline(g, dual, gpu_ms):
    """O3 (the wedge oracle: Sec. IV-B's alternative algorithm with an exact
    counter, degree pruning of Sec. IV-C) over every row of the workload at
    s = 8 and 16: 16 threads (median of 3), and one thread at s = 16 (once).
    `gpu_ms` maps s to the GPU's build time for the same builds."""
    import oracle

    P = oracle.prepare(g.row_ptr, g.col, g.n_edges, g.n_vertices, dual=dual)
    threads = oracle_threads()
    s_set = (8, 16) if not dual else (8, 32)
    per_s = {}
    total = 0.0
    for s in s_set:
        t, st = time_oracle(P, s, threads, 3)
        per_s[str(s)] = {"s": t, "pairs": st.n_pairs, "wedges": st.wedges}
        total += t
        log(f"CPU oracle s={s}: {t:.2f} s on {threads} threads")
    t1, _ = time_oracle(P, s_set[-1], 1, 1)
    log(f"CPU oracle s={s_set[-1]}: {t1:.2f} s on 1 thread")
    value = len(s_set) * g.nnz / total
    gpu_same = sum(gpu_ms[s] for s in s_set if s in gpu_ms)
    return {"value": value, "unit": "incidence entries/s", "cores": threads, "kind": "oracle",
            "sample": f"O3 wedge oracle over every row of the whole workload, s in {list(s_set)} "
                      f"(2 of the step's builds), {threads} threads, median of 3; measured, "
                      f"not extrapolated",
            "cpu_model": cpu_model(), "per_s_seconds": per_s,
            "one_thread": {"s": s_set[-1], "seconds": t1,
                           "entries_per_s": g.nnz / t1},
            "gpu_same_builds_entries_per_s": (len(s_set) * g.nnz / (gpu_same / 1e3)
                                              if gpu_same > 0 else None)}


def cpu_full(g):
    """The oracle over the whole sweeps (every s of the primal and the dual
    step, every row): 16 threads median of 3, one thread once.  Printed as its
    own JSON line."""
    import oracle

    gen = gen_mod()
    threads = oracle_threads()
    res = {"form": "cpu", "cpu_model": cpu_model(), "threads": threads, "nnz": g.nnz}
    for dual, s_list in ((0, gen.POWERLAW_S), (1, gen.DUAL_S)):
        P = oracle.prepare(g.row_ptr, g.col, g.n_edges, g.n_vertices, dual=dual)
        side = {"per_s": {}}
        tn = t1 = 0.0
        for s in s_list:
            t, st = time_oracle(P, s, threads, 3)
            u, _ = time_oracle(P, s, 1, 1)
            log(f"CPU oracle dual={dual} s={s}: {t:.2f} s on {threads} threads, "
                f"{u:.2f} s on 1 thread")
            side["per_s"][str(s)] = {"threads_s": t, "one_thread_s": u, "pairs": st.n_pairs,
                                     "wedges": st.wedges}
            tn += t
            t1 += u
        side.update({"sweep_s": tn, "sweep_one_thread_s": t1,
                     "entries_per_s": len(s_list) * g.nnz / tn,
                     "entries_per_s_one_thread": len(s_list) * g.nnz / t1})
        res["dual" if dual else "primal"] = side
    print(json.dumps(res), flush=True)


def gen_mod():
    from paper_2010_11448_amd import gen

    return gen


def kernel_sha():
    h = hashlib.sha256()
    for src in KERNEL_SRCS:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(form):
    """HBM bytes per launch of the task kernel from the committed counter
    summary, if it was taken on the current kernel source and this form
    (form None: no summary applies, e.g. the product route)."""
    if form is None:
        return None
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


# ------------------------------------------------------------- workloads

def draw_workloads(args, need_batch, need_serve):
    """Every synthetic graph the run needs, drawn in worker processes before
    the GPU is touched."""
    gen = gen_mod()
    specs = [("powerlaw_1m", (), {"scale": args.scale})]
    nb = args.graphs if need_batch else 0
    specs += [("batch_graph", (g,), {}) for g in range(nb)]
    ns, nl = (args.catalog_small, args.catalog_large) if need_serve else (0, 0)
    # serving catalog: batch-law graphs under their own seed, and power-law
    # graphs of the full size with seeds following the timed graph's
    specs += [("batch_graph", (g,), {"seed": gen.SERVE_SEED}) for g in range(ns)]
    specs += [("powerlaw_1m", (), {"seed": gen.POWERLAW_SEED + 1 + i}) for i in range(nl)]
    t0 = time.perf_counter()
    graphs = gen.make_many(specs, workers=max(1, args.gen_workers))
    log(f"drew {len(graphs)} graphs in {time.perf_counter() - t0:.1f} s")
    g = graphs[0]
    g.meta.setdefault("workload", "powerlaw_1Mx2M" if args.scale == 1.0 else "powerlaw_scaled")
    batch = graphs[1:1 + nb]
    catalog = graphs[1 + nb:]
    return g, batch, catalog


# ------------------------------------------------------------ plain form

def bench_plain(args, g, dual, s_list, dev):
    import torch

    from paper_2010_11448_amd import sline

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
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    torch.cuda.empty_cache()
    ms_per_step = (t1 - t0) * 1000.0 / max(args.steps, 1)
    value = len(s_list) * g.nnz / (ms_per_step / 1000.0)

    alg_bytes = 0.0
    task_ms = 0.0
    launches = 0
    build_bytes = 0.0
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
        # the whole build under the per-(graph, s) algorithmic bytes
        bb = 12.0 * st["nnz_kept"] + 4.0 * st["wedges"] + 12.0 * st["n_pairs"]
        build_bytes += bb
        med = lambda k: float(np.median([r[1][k] for r in recs]))
        builds[str(s)] = {
            "p50_ms": pct(times, 50), "p99_ms": pct(times, 99),
            "pairs": st["n_pairs"], "wedges": st["wedges"], "kept_items": st["n_kept"],
            "build_alg_bytes": bb, "build_GBps": bb / 1e6 / max(pct(times, 50), 1e-9),
            "task_kernel_alg_bytes": b, "ms_tasks": med("ms_tasks"),
            "task_kernel_GBps": b / 1e6 / max(med("ms_tasks"), 1e-9),
            "ms_transpose": med("ms_transpose"), "ms_prepare": med("ms_prepare"),
            "ms_count": med("ms_count"), "ms_scan": med("ms_scan"), "ms_fill": med("ms_fill"),
            "heavy_items": st["n_heavy"], "small_items": st["n_small"], "passes": st["passes"],
            "product_nnz": st["product_nnz"], "ms_product": st["ms_product"],
            "ms_filter": st["ms_filter"],
        }
    achieved = alg_bytes / 1e9 / (task_ms / 1000.0) if task_ms > 0 else 0.0
    form = None if args.spgemm else args.form
    tr = committed_traffic(form if args.scale == 1.0 and not args.s else None)
    traffic = tr["bytes_per_launch"] if tr else None
    build_GBps = build_bytes / 1e9 / (ms_per_step / 1000.0)
    line = {
        "metric": METRIC,
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
                     "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT) if tr else None,
                     "build_GBps": build_GBps, "build_frac": build_GBps / HBM_PEAK_GBS,
                     "build_alg_bytes": "12*nnz_s + 4*W_s + 12*|L_s| per build, whole step"},
        "builds": builds,
    }
    gpu_ms = {s: builds[str(s)]["p50_ms"] for s in s_list}
    return line, gpu_ms


# ---------------------------------------------------------- uniform form

def bench_uniform(dev, reps=5):
    """The 2,000 x 5,000 uniform workload, s = 1..8, seeds 11, 12, 13: one
    plain build per (seed, s), latency-bound."""
    import torch

    from paper_2010_11448_amd import gen, sline

    ctx = sline.Context(0)
    out = {"workload": "uniform_2000x5000", "s": list(gen.UNIFORM_S), "seeds": list(gen.UNIFORM_SEEDS)}
    lat = []
    nnz_total = 0
    t_total = 0.0
    pairs = {}
    for seed in gen.UNIFORM_SEEDS:
        h = gen.uniform_2000(seed)
        rp = torch.from_numpy(h.row_ptr).to(dev)
        col = torch.from_numpy(h.col).to(dev)
        for s in gen.UNIFORM_S:
            L = ctx.build(rp, col, h.n_vertices, s, 0)  # warm
            pairs[f"{seed}/{s}"] = len(L)
            del L
        torch.cuda.synchronize()
        for _ in range(reps):
            t0 = time.perf_counter()
            for s in gen.UNIFORM_S:
                tb = time.perf_counter()
                L = ctx.build(rp, col, h.n_vertices, s, 0)
                lat.append((time.perf_counter() - tb) * 1e3)
                del L
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            nnz_total += len(gen.UNIFORM_S) * h.nnz
    ctx.close()
    out.update({"entries_per_s": nnz_total / t_total, "build_p50_ms": pct(lat, 50),
                "build_p99_ms": pct(lat, 99), "builds": len(lat), "pairs": pairs})
    return out


# ------------------------------------------------------------ batch form

def bench_batch(args, graphs_h, dev, steps, warmup):
    """Batched form: one sline_build_batch call vs one sline_build call per
    graph, same graphs, same GPU, both with library-allocated results."""
    import torch

    from paper_2010_11448_amd import autotune, sline

    s_list = [int(h.meta["s"]) for h in graphs_h]  # each graph's own s, drawn with it
    dual = [0] * len(graphs_h)
    graphs = [(torch.from_numpy(h.row_ptr).to(dev), torch.from_numpy(h.col).to(dev),
               h.n_vertices) for h in graphs_h]
    nnz = sum(h.nnz for h in graphs_h)
    ctx = sline.Context(0)
    flags = sline.SLINE_PROFILE

    def run_batch():
        outs = ctx.build_batch_owned(graphs, s_list, dual, flags)
        ctx.free_edges(outs, len(graphs))

    def run_plain():
        for (rp, col, nv), s, d in zip(graphs, s_list, dual):
            out = ctx.build_owned(rp, col, nv, s, d, flags)
            ctx.free_edges([out])

    tuned, source = None, "defaults"
    sig = autotune.batch_signature(graphs, s_list, dual)
    if args.autotune:
        log("autotuning on the batch")
        tuned, secs = autotune.tune(ctx, run_batch, budget_s=args.tune_budget,
                                    log=lambda m: print(m, file=sys.stderr, flush=True))
        source = "autotuned"
        if args.tune_cache:
            autotune.save_cached(args.tune_cache, sig, tuned, secs)
    elif args.tune_cache:
        entry = autotune.load_cached(args.tune_cache, sig)
        if entry:
            ctx.set_tuning(**entry)
            tuned, source = ctx.tuning(), f"cache {os.path.relpath(args.tune_cache, HERE)}"
    for _ in range(max(warmup, 1)):
        run_batch()
        run_plain()
    torch.cuda.synchronize()
    tb = []
    for i in range(steps):
        t0 = time.perf_counter()
        run_batch()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        log(f"batch step {i + 1}/{steps} {tb[-1] * 1e3:.1f} ms")
    st = ctx.stats()
    tp = []
    for i in range(steps):
        t0 = time.perf_counter()
        run_plain()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
        log(f"plain step {i + 1}/{steps} {tp[-1] * 1e3:.1f} ms")
    # the same batch as a plan: sized once, then replayed as one graph launch
    # with the results left in the plan's arrays
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = sline.BatchPlan(ctx, graphs, s_list, dual)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    plan_bytes, plan_tasks, plan_pairs = plan.info()
    for _ in range(max(warmup, 1)):
        plan.run_raw()
    tr = []
    for i in range(steps):
        t0 = time.perf_counter()
        rc = plan.run_raw()
        tr.append(time.perf_counter() - t0)
        if rc != sline.SLINE_OK:
            raise sline.SlineError(rc, sline.sline_last_error(ctx.ctx))
        log(f"plan replay {i + 1}/{steps} {tr[-1] * 1e3:.1f} ms")
    plan_pairs_run = int(ctx.stats()["n_pairs"])
    plan.close()
    ctx.close()
    t_batch = sum(tb) / len(tb)
    t_plain = sum(tp) / len(tp)
    t_plan = sum(tr) / len(tr)
    b = 12.0 * st["heavy_nnz"] + 4.0 * st["heavy_wedges"] + 8.0 * st["heavy_pairs"]
    ach = b / 1e9 / (st["ms_tasks"] / 1e3) if st["ms_tasks"] > 0 else 0.0
    return {
        "workload": f"batch_lognormal_{len(graphs_h)}", "graphs": len(graphs_h), "nnz": nnz,
        "items": sum(h.n_edges for h in graphs_h), "s": "per graph, uniform on 1..12",
        "batched_entries_per_s": nnz / t_batch, "plain_entries_per_s": nnz / t_plain,
        "batched_vs_plain": t_plain / t_batch,
        "batched_ms_p50": pct([x * 1e3 for x in tb], 50),
        "batched_ms_p99": pct([x * 1e3 for x in tb], 99),
        "plain_ms_p50": pct([x * 1e3 for x in tp], 50),
        "plain_ms_p99": pct([x * 1e3 for x in tp], 99),
        "steps": steps, "pairs": st["n_pairs"], "tuning": tuned or None,
        "tuning_source": source, "tuning_class": sig,
        "batched_stage_ms": {k: st[k] for k in ("ms_transpose", "ms_prepare", "ms_count",
                                                "ms_scan", "ms_fill", "ms_tasks")},
        "task_kernel_GBps": ach,
        "plan": {"replay_ms_p50": pct([x * 1e3 for x in tr], 50),
                 "replay_ms_p99": pct([x * 1e3 for x in tr], 99),
                 "replay_vs_batched": t_batch / t_plan, "replay_vs_plain": t_plain / t_plan,
                 "create_ms": t_create * 1e3, "device_bytes": plan_bytes,
                 "task_capacity": plan_tasks, "pair_capacity": plan_pairs,
                 "pairs": plan_pairs_run},
    }


# ------------------------------------------------------------ serve form

def bench_serve(args, catalog, dev):
    """Serving form: Poisson arrivals through the query loop; the same queries
    at saturation (all submitted at once); and the same queries with one plain
    call each."""
    import torch

    from paper_2010_11448_amd import gen, sline

    ns, nl = args.catalog_small, args.catalog_large
    # the server maps its own device memory: hand back what torch's caching
    # allocator still holds from the forms timed before
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    dgr = [(torch.from_numpy(h.row_ptr).to(dev), torch.from_numpy(h.col).to(dev), h.n_vertices)
           for h in catalog]
    qs = gen.serving_arrivals(ns, nl, rate=args.rate, duration_s=args.duration)
    srv = sline.Server(0, hbm_budget_bytes=int(args.budget_gb * (1 << 30)), max_batch=64,
                       workers=args.workers)
    srv.set_reuse(int(args.reuse_gb * (1 << 30)), REUSE_MIN_NNZ, lookahead=True)
    ids = [srv.register(rp, col, n) for rp, col, n in dgr]
    # warm the server: a few queries, and the largest result of each large
    # graph (maps the device memory its cache will reuse)
    warm = [(ids[q.graph_id], q.s, q.dual) for q in qs[:8]]
    warm += [(ids[ns + i], 1, 0) for i in range(min(nl, 2))]
    for gid, s_, d_ in warm:
        t = srv.submit(gid, s_, d_)
        while srv.poll(t, keep=False) is None:
            time.sleep(0.0005)
    log(f"serving {len(qs)} queries over {args.duration:.0f} s")
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
            log(f"served {len(infos)}/{len(qs)} (submitted {k}, queued {qd}, running batches {rn})")
        if k < len(qs):
            time.sleep(max(0.0, min(0.0005, qs[k].arrival_s - (time.perf_counter() - t0))))
        else:
            time.sleep(0.0002)
    wall = time.perf_counter() - t0
    lat = [(infos[i]["t_done_ns"] - infos[i]["t_submit_ns"]) / 1e6 for i in range(len(qs))]
    nnz = sum(catalog[q.graph_id].nnz for q in qs)
    batch_sizes = [infos[i]["batch_size"] for i in range(len(qs))]
    first = min(infos[i]["t_submit_ns"] for i in range(len(qs)))
    last = max(infos[i]["t_done_ns"] for i in range(len(qs)))
    reuse_arrival = srv.reuse_stats()

    def saturate():
        t1 = time.perf_counter()
        ts = [srv.submit(ids[q.graph_id], q.s, q.dual) for q in qs]
        while ts:
            ts = [t for t in ts if srv.poll(t, keep=False) is None]
            if ts:
                time.sleep(0.0002)
        return time.perf_counter() - t1

    # saturation: every query at once, first without result reuse, then with
    # it starting from nothing kept
    log("saturation without result reuse")
    srv.set_reuse(0)
    t_sat_plain_server = saturate()
    log("saturation with result reuse")
    srv.set_reuse(int(args.reuse_gb * (1 << 30)), REUSE_MIN_NNZ, lookahead=True)
    r0 = srv.reuse_stats()
    t_sat = saturate()
    r1 = srv.reuse_stats()
    srv.close()
    log("plain calls, one per query")
    torch.cuda.empty_cache()
    ctx = sline.Context(0)
    # the server reserved its memory before its timing began: the plain side
    # gets the same, one untimed pass over the full-size queries (the ones
    # whose workspaces and results need fresh device memory)
    for q in qs:
        if q.graph_id >= ns:
            rp, col, n = dgr[q.graph_id]
            ctx.free_edges([ctx.build_owned(rp, col, n, q.s, q.dual)])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    t_plain_large = 0.0
    for q in qs:
        rp, col, n = dgr[q.graph_id]
        tq = time.perf_counter()
        out = ctx.build_owned(rp, col, n, q.s, q.dual)
        ctx.free_edges([out])
        if q.graph_id >= ns:
            torch.cuda.synchronize()
            t_plain_large += time.perf_counter() - tq
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t2
    ctx.close()
    large = [lat[i] for i, q in enumerate(qs) if q.graph_id >= ns]
    slowest = sorted(range(len(qs)), key=lambda i: -lat[i])[:8]
    slow = [{"ms": lat[i], "large": qs[i].graph_id >= ns, "s": qs[i].s, "dual": qs[i].dual,
             "batch": infos[i]["batch_size"],
             "wait_ms": (infos[i]["t_start_ns"] - infos[i]["t_submit_ns"]) / 1e6} for i in slowest]
    small = [lat[i] for i, q in enumerate(qs) if q.graph_id < ns]
    return {
        "workload": f"serving_poisson{args.rate:.0f}_{args.duration:.0f}s",
        "queries": len(qs), "catalog_small": ns, "catalog_large": nl,
        "budget_gb": args.budget_gb, "workers": args.workers, "duration_s": args.duration,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": max(lat),
        "small_p50_ms": pct(small, 50), "small_p99_ms": pct(small, 99),
        "large_queries": len(large), "large_p50_ms": pct(large, 50), "large_p99_ms": pct(large, 99),
        "queries_per_s_arrival_run": len(qs) / ((last - first) / 1e9),
        "entries_per_s_arrival_run": nnz / ((last - first) / 1e9),
        "wall_s": wall, "mean_batch": sum(batch_sizes) / len(batch_sizes),
        "max_batch": max(batch_sizes),
        "saturation_s": t_sat, "saturation_queries_per_s": len(qs) / t_sat,
        "saturation_entries_per_s": nnz / t_sat,
        "plain_s": t_plain, "plain_large_s": t_plain_large,
        "plain_queries_per_s": len(qs) / t_plain,
        "served_vs_plain": t_plain / t_sat,
        "saturation_no_reuse_s": t_sat_plain_server,
        "served_vs_plain_no_reuse": t_plain / t_sat_plain_server,
        "slowest": slow,
        "reuse": {"cache_bytes": int(args.reuse_gb * (1 << 30)), "min_nnz": REUSE_MIN_NNZ,
                  "lookahead": True,
                  "arrival_run_reused": reuse_arrival["reused"],
                  "saturation_reused": r1["reused"] - r0["reused"],
                  "saturation_kept": r1["kept"] - r0["kept"]},
    }


# ----------------------------------------------------------- stages form

def _timed_ms(fn, reps=3):
    import torch

    ts = []
    out = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
        if reps > 1:
            del out
            out = None
    return float(np.median(ts)), out


def bench_stages(g, dev, variant_scale=0.05, variant_s=(2, 4, 6, 8)):
    """The rows after L_s on the 1,000,000 x 2,000,000 workload: the s-sweep
    (count the smallest s, filter the rest) against plain builds, squeezing
    and components per s, relabel-by-degree both ways, and the variants f0..f4
    of Table III on the same law at `variant_scale` (the variants without
    visited skipping make a set intersection per wedge), with the oracle's
    heuristic algorithm (O2) timed on the host for the same variants."""
    import torch

    import oracle
    from paper_2010_11448_amd import gen, sline

    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    ctx = sline.Context(0)
    out = {}
    s_list = list(gen.POWERLAW_S)
    ctx.build_sweep(rp, col, g.n_vertices, s_list, 0)  # warm
    t_sweep, _ = _timed_ms(lambda: ctx.build_sweep(rp, col, g.n_vertices, s_list, 0))
    plain = {}
    for s in s_list:
        plain[s], _ = _timed_ms(lambda: ctx.build(rp, col, g.n_vertices, s, 0))
    torch.cuda.empty_cache()
    L1 = ctx.build(rp, col, g.n_vertices, 1, 0)
    t_filter, L2 = _timed_ms(lambda: ctx.filter(L1, 2), reps=1)
    filt_bytes = 16.0 * len(L1) + 12.0 * len(L2)  # w twice, a and b once; kept pairs written
    del L1, L2
    torch.cuda.empty_cache()
    out["sweep"] = {"s": s_list, "sweep_ms": t_sweep, "plain_ms_sum": sum(plain.values()),
                    "plain_ms": {str(k): v for k, v in plain.items()},
                    "sweep_vs_plain": sum(plain.values()) / t_sweep,
                    "filter_l1_to_l2_ms": t_filter,
                    "filter_GBps": filt_bytes / 1e6 / t_filter}
    log(f"stages: sweep {t_sweep:.1f} ms vs plain {sum(plain.values()):.1f} ms")
    per_s = {}
    for s in s_list:
        L = ctx.build(rp, col, g.n_vertices, s, 0)
        rec = {"pairs": len(L)}
        if len(L) < (1 << 31) - 1:
            rec["squeeze_ms"], G = _timed_ms(lambda: ctx.squeeze(L, g.n_edges), reps=1)
            rec["nodes"] = G["n_nodes"]
            del G
        rec["components_ms"], (comp, ncomp) = _timed_ms(lambda: ctx.components(L, g.n_edges),
                                                        reps=1)
        rec["components"] = ncomp
        rec["build_ms"] = plain[s]
        per_s[str(s)] = rec
        del L, comp
        torch.cuda.empty_cache()
        log(f"stages: s={s} {rec}")
    out["squeeze_components"] = per_s
    rel = {}
    for name, flag in (("asc", sline.SLINE_RELABEL_ASC), ("desc", sline.SLINE_RELABEL_DESC)):
        rel[name] = {}
        for s in (2, 4, 8, 16):
            t, _ = _timed_ms(lambda: ctx.build(rp, col, g.n_vertices, s, 0, flag), reps=2)
            rel[name][str(s)] = t
        log(f"stages: relabel {name} {rel[name]}")
    rel["plain"] = {str(s): plain[s] for s in (2, 4, 8, 16)}
    out["relabel_ms"] = rel
    torch.cuda.empty_cache()
    # variants f0..f4 on a smaller graph of the same law
    h = gen.powerlaw_1m(scale=variant_scale)
    hr = torch.from_numpy(h.row_ptr).to(dev)
    hc = torch.from_numpy(h.col).to(dev)
    threads = oracle_threads()
    var = {"workload": h.meta.get("workload"), "n_edges": h.n_edges, "nnz": h.nnz,
           "s": list(variant_s), "cpu_threads": threads, "gpu_ms": {}, "cpu_o2_ms": {},
           "intersections": {}}
    for v in ("f0", "f1", "f2", "f3", "f4"):
        fl = sline.VARIANT_FLAGS[v]
        var["gpu_ms"][v] = {}
        var["cpu_o2_ms"][v] = {}
        var["intersections"][v] = {}
        for s in variant_s:
            ctx.build(hr, hc, h.n_vertices, s, 0, fl)
            t, _ = _timed_ms(lambda: ctx.build(hr, hc, h.n_vertices, s, 0, fl), reps=2)
            var["gpu_ms"][v][str(s)] = t
            t0 = time.perf_counter()
            _, ost = oracle.alg_h(h.row_ptr, h.col, h.n_edges, h.n_vertices, s,
                                  variant=oracle.VARIANTS[v], threads=threads, keep=False)
            var["cpu_o2_ms"][v][str(s)] = (time.perf_counter() - t0) * 1e3
            var["intersections"][v][str(s)] = ost.intersections
        log(f"stages: variant {v} gpu {var['gpu_ms'][v]} cpu {var['cpu_o2_ms'][v]}")
    out["variants"] = var
    ctx.close()
    return out


METRIC = "s-line graph build: incidence entries/s, % HBM peak; batched vs plain; p50/p99"
# serving: device bytes of kept results that answer later queries by a filter
REUSE_BYTES = 96 << 30
REUSE_MIN_NNZ = 1 << 20


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rows of the result shard across GPUs without exchange)",
              file=sys.stderr)
        sys.exit(2)
    if args.form == "cpu":
        g, _, _ = draw_workloads(args, False, False)
        cpu_full(g)
        return
    sub = args.form == "plain" and not args.plain_only and args.scale == 1.0 and not args.s
    need_batch = sub or args.form == "batch"
    need_serve = sub or args.form == "serve"
    # every graph is drawn before the GPU is touched (worker processes)
    g, batch_h, catalog = draw_workloads(args, need_batch, need_serve)
    import torch

    if args.form == "copy":
        copy_calibration(max(args.steps, 1))
        return
    dev = torch.device("cuda", 0)
    if args.form == "batch":
        res = bench_batch(args, batch_h, dev, args.steps, args.warmup)
        print(json.dumps({"metric": METRIC, "value": res["batched_entries_per_s"],
                          "unit": "incidence entries/s", "n_gpus": 1,
                          "ms_per_step": res["batched_ms_p50"], "config": {"workload": res["workload"]},
                          "batch": res}), flush=True)
        return
    if args.form == "stages":
        print(json.dumps({"form": "stages", "stages": bench_stages(g, dev)}), flush=True)
        return
    if args.form == "serve":
        res = bench_serve(args, catalog, dev)
        print(json.dumps({"metric": METRIC, "value": res["saturation_entries_per_s"],
                          "unit": "incidence entries/s", "n_gpus": 1,
                          "config": {"workload": res["workload"]}, "serve": res}), flush=True)
        return
    gen = gen_mod()
    dual = 1 if args.form == "dual" else 0
    s_list = tuple(int(x) for x in args.s.split(",")) if args.s else (
        gen.DUAL_S if dual else gen.POWERLAW_S)
    line, gpu_ms = bench_plain(args, g, dual, s_list, dev)
    if sub:
        log("uniform 2000 x 5000 workload")
        line["uniform"] = bench_uniform(dev)
        log(f"batch of {len(batch_h)} graphs")
        line["batch"] = bench_batch(args, batch_h, dev, args.batch_steps, 1)
        del batch_h
        log("serving")
        line["serve"] = bench_serve(args, catalog, dev)
        log("stages after L_s")
        line["stages"] = bench_stages(g, dev)
    if not args.no_cpu_baseline and not args.spgemm:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(g, dual, gpu_ms)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
