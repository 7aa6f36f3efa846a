"""The autotuner's search and cache, driven by a stand-in context whose cost
depends on the launch parameters (no GPU)."""

from __future__ import annotations

import time

from paper_2010_11448_amd import autotune


class FakeCtx:
    def __init__(self):
        self.t = {"small_max_wedges": 512, "task_wedges": 5000, "group_parts": 8, "light_len": 8,
                  "small_grid_per_cu": 16, "task_grid_per_cu": 4, "stage_max_bytes": 1 << 30}

    def tuning(self):
        return dict(self.t)

    def set_tuning(self, **kw):
        assert set(kw) == set(self.t)
        self.t = dict(kw)


def test_coordinate_descent_finds_the_cheap_setting():
    ctx = FakeCtx()
    best_tw, best_gp = 10000, 32

    def run():
        t = ctx.t
        cost = 0.002 + 0.004 * (t["task_wedges"] != best_tw) + 0.004 * (t["group_parts"] != best_gp)
        time.sleep(cost)

    space = {"task_wedges": [2500, 5000, 10000], "group_parts": [8, 16, 32]}
    tuned, secs = autotune.tune(ctx, run, space=space, rounds=2, budget_s=30)
    assert tuned["task_wedges"] == best_tw and tuned["group_parts"] == best_gp
    assert ctx.t == tuned
    assert secs < 0.006


def test_budget_stops_the_search_and_keeps_a_valid_setting():
    ctx = FakeCtx()
    tuned, _ = autotune.tune(ctx, lambda: time.sleep(0.01), space=autotune.SPACE, budget_s=0.0)
    assert tuned == ctx.t and tuned["task_wedges"] == 5000


def test_signature_and_cache(tmp_path):
    sig = autotune.signature([1000, 3000], [1, 5], [0, 1])
    assert sig == autotune.signature([1000, 3000], [2, 9], [1, 0])
    assert sig != autotune.signature([10 ** 8], [1], [0])
    path = str(tmp_path / "tune.json")
    assert autotune.load_cached(path, sig) is None
    autotune.save_cached(path, sig, {"task_wedges": 7000}, 0.5)
    assert autotune.load_cached(path, sig) == {"task_wedges": 7000}


class _Col:
    def __init__(self, n):
        self.n = n

    def numel(self):
        return self.n


def test_cached_tuning_applies_and_restores(tmp_path):
    """The batch path's use of the cache: the entry for the batch's class
    applies inside the block, the context's own tuning comes back after, and
    a missing file or entry changes nothing."""
    ctx = FakeCtx()
    graphs = [(None, _Col(1000), 5), (None, _Col(3000), 7)]
    sig = autotune.batch_signature(graphs, [1, 5], [0, 1])
    assert sig == autotune.signature([1000, 3000], [1, 5], [0, 1])
    path = str(tmp_path / "tune.json")
    before = ctx.tuning()
    with autotune.cached_tuning(ctx, path, sig) as entry:
        assert entry is None and ctx.tuning() == before
    autotune.save_cached(path, sig, {"task_wedges": 7000, "group_parts": 16}, 0.5)
    with autotune.cached_tuning(ctx, path, sig) as entry:
        assert entry == {"task_wedges": 7000, "group_parts": 16}
        assert ctx.tuning() == {**before, "task_wedges": 7000, "group_parts": 16}
    assert ctx.tuning() == before
    other = autotune.signature([10 ** 8], [1], [0])
    with autotune.cached_tuning(ctx, path, other) as entry:
        assert entry is None and ctx.tuning() == before
    with autotune.cached_tuning(ctx, None, sig) as entry:
        assert entry is None and ctx.tuning() == before


def test_cached_tuning_skips_what_the_context_refuses(tmp_path):
    """An entry's parameters the context does not have are left out, and an
    entry whose values the context refuses is not applied: the call goes on
    with the context's own tuning."""

    class Strict(FakeCtx):
        def set_tuning(self, **kw):
            if kw["task_wedges"] < 64:
                raise ValueError("tuning value out of range")
            super().set_tuning(**kw)

    ctx = Strict()
    path = str(tmp_path / "tune.json")
    sig = autotune.signature([1000], [1], [0])
    before = ctx.tuning()
    autotune.save_cached(path, sig, {"task_wedges": 7000, "not_a_parameter": 32}, 0.5)
    with autotune.cached_tuning(ctx, path, sig) as entry:
        assert entry == {"task_wedges": 7000}
        assert ctx.tuning() == {**before, "task_wedges": 7000}
    assert ctx.tuning() == before
    autotune.save_cached(path, sig, {"task_wedges": 1}, 0.5)
    with autotune.cached_tuning(ctx, path, sig) as entry:
        assert entry is None and ctx.tuning() == before
    assert ctx.tuning() == before
