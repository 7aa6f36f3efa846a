"""Autotuner for the launch parameters of the counting stage.

The parameters (``sline_tuning``) change speed, never the result: task size
in wedges, parts per workgroup group, the one-wave / workgroup split, the
lane-walk threshold, the resident grid sizes and the LDS table sizes of the
two counting kernels.  ``tune`` measures a
workload (any callable that runs builds on a Context) under candidate
settings by coordinate descent -- one parameter at a time, keeping the best
value before moving to the next -- within a time budget.  Results can be kept
in a JSON cache keyed by a coarse workload signature, so a later run on a
workload of the same class uses the tuned setting: ``Context.build_batch``,
``Context.build_batch_owned`` and ``BatchPlan`` take the cache's path
(``tuning_cache``) and apply its entry for their batch around the call.
"""

from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Iterable

SPACE: dict[str, list[int]] = {
    "task_wedges": [2500, 3500, 5000, 7000, 10000, 14000],
    "group_parts": [2, 4, 8, 16, 32],
    "small_slots": [512, 1024, 2048],
    "task_slots": [4480, 8960, 13440, 17920],
    "tiny_max_wedges": [0, 4, 10],
    "small_max_wedges": [0, 128, 256, 512, 1024],
    "light_len": [2, 4, 8, 12, 16],
    "small_grid_per_cu": [4, 8, 16, 32],
    "task_grid_per_cu": [2, 3, 4],
    "dense_min_wedges": [0, 1024, 4096, 16384],
}


def signature(nnz: Iterable[int], s: Iterable[int], dual: Iterable[int]) -> str:
    """Workload class: log2 buckets of total incidences and graph count, and
    the share of each side and of small s."""
    nnz = list(nnz)
    s = list(s)
    dual = list(dual)
    tot = max(sum(nnz), 1)
    g = max(len(nnz), 1)
    small_s = sum(1 for x in s if x <= 2) / max(len(s), 1)
    d = sum(dual) / max(len(dual), 1)
    return f"nnz2^{int(math.log2(tot))}-g2^{int(math.log2(g))}-s12:{small_s:.1f}-dual:{d:.1f}"


def _sync() -> None:
    import torch

    if torch.cuda.is_available():
        torch.cuda.synchronize()


def _timed(ctx, run: Callable[[], None], reps: int) -> float:
    best = float("inf")
    for _ in range(reps):
        _sync()
        t0 = time.perf_counter()
        run()
        _sync()
        best = min(best, time.perf_counter() - t0)
    return best


def tune(ctx, run: Callable[[], None], space: dict[str, list[int]] | None = None,
         rounds: int = 2, reps: int = 1, budget_s: float = 60.0, log=None) -> tuple[dict, float]:
    """Coordinate descent over ``space``; returns (best tuning dict, seconds)."""
    space = space or SPACE
    start = time.perf_counter()
    best = ctx.tuning()
    run()  # warm caches and workspaces
    best_t = _timed(ctx, run, reps)
    if log:
        log(f"autotune: base {best} {best_t * 1e3:.1f} ms")
    for _ in range(rounds):
        improved = False
        for key, values in space.items():
            for v in values:
                if time.perf_counter() - start > budget_s:
                    ctx.set_tuning(**best)
                    return best, best_t
                if v == best[key]:
                    continue
                cand = {**best, key: v}
                try:
                    ctx.set_tuning(**cand)
                except RuntimeError:
                    # a combination the library refuses (small_max_wedges
                    # above half the one-wave table)
                    ctx.set_tuning(**best)
                    continue
                t = _timed(ctx, run, reps)
                if log:
                    log(f"autotune: {key}={v} {t * 1e3:.1f} ms")
                if t < best_t * 0.98:
                    best, best_t, improved = cand, t, True
            ctx.set_tuning(**best)
        if not improved:
            break
    ctx.set_tuning(**best)
    return best, best_t


def batch_signature(graphs, s, dual=None) -> str:
    """``signature`` of a batch of (row_ptr, col, n_vertices) device tensors
    (the incidences of a graph are the length of its col)."""
    nnz = [int(col.numel()) for _, col, _ in graphs]
    return signature(nnz, s, list(dual) if dual is not None else [0] * len(nnz))


class cached_tuning:
    """Inside the block, ``ctx`` runs with the tuning stored for ``sig`` in the
    cache file at ``path`` (merged over its own); its own tuning comes back on
    exit.  No file, no entry or ``path`` None: nothing changes.  The cache is a
    speed hint, never a reason for a call to fail: parameters the context does
    not have are left out, and an entry the context refuses (a value outside
    its ranges) is not applied.  The value of the block is the applied entry,
    or None."""

    def __init__(self, ctx, path: str | None, sig: str):
        self.ctx, self.path, self.sig = ctx, path, sig
        self.prev = None

    def __enter__(self):
        entry = load_cached(self.path, self.sig) if self.path else None
        if not entry:
            return None
        prev = self.ctx.tuning()
        entry = {k: v for k, v in entry.items() if k in prev}
        try:
            self.ctx.set_tuning(**{**prev, **entry})
        except Exception:
            self.ctx.set_tuning(**prev)
            return None
        self.prev = prev
        return entry

    def __exit__(self, *exc):
        if self.prev is not None:
            self.ctx.set_tuning(**self.prev)
        return False


def load_cached(path: str, sig: str) -> dict | None:
    try:
        with open(path) as f:
            return json.load(f).get(sig, {}).get("tuning")
    except (OSError, ValueError):
        return None


def save_cached(path: str, sig: str, tuning: dict, seconds: float) -> None:
    data = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
    data[sig] = {"tuning": tuning, "seconds": seconds}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
