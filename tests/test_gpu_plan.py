"""Batch plans: a batch sized once and replayed as one HIP graph launch.

Bar: bit-exact -- every replay returns, for every graph, the oracle's L_s of
that graph as its arrays hold it at the time of the run, at the run's s; a
run whose input or work outgrows the plan fails with the documented status
and leaves the plan usable.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2010_11448_amd import gen

from helpers import assert_same, to_device
from test_gpu_batch import _mixed_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2010_11448_amd import sline

    assert torch.cuda.is_available()
    c = sline.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def dev():
    import torch

    return torch.device("cuda", 0)


def _plan(ctx, dg, graphs, ss, duals, flags=0):
    from paper_2010_11448_amd import sline

    return sline.BatchPlan(ctx, [(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)],
                           ss, duals, flags)


def _host(L):
    """A device result as host arrays, the form assert_same compares with."""
    from types import SimpleNamespace

    return SimpleNamespace(a=L.a.cpu().numpy(), b=L.b.cpu().numpy(), w=L.w.cpu().numpy())


def _check(res, graphs, ss, duals, what):
    assert len(res) == len(graphs)
    for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
        ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
        assert_same(res[g], ref, f"{what}: graph {g} s={s} dual={d}")


@pytest.mark.parametrize("seed", [3, 7])
def test_plan_replays_equal_the_oracle(ctx, dev, seed):
    graphs, ss, duals = _mixed_batch(24, seed)
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: plan seed={seed} s={ss} dual={duals}", flush=True)
    plan = _plan(ctx, dg, graphs, ss, duals)
    try:
        nbytes, tcap, pcap = plan.info()
        assert nbytes > 0 and tcap >= 1 and pcap >= 1
        first = plan.run(copy=True)
        _check(first, graphs, ss, duals, "first run")
        assert pcap == max(sum(len(r) for r in first), 1)
        # a second replay recomputes the same result in the same arrays
        again = plan.run()
        for g in range(len(graphs)):
            assert_same(again[g], _host(first[g]), f"replay graph {g}")
        # and equals the eager batched build
        eager = ctx.build_batch([(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)],
                                ss, duals)
        for g in range(len(graphs)):
            assert_same(again[g], _host(eager[g]), f"eager graph {g}")
    finally:
        plan.close()


def test_plan_runs_at_larger_s(ctx, dev):
    graphs, ss, duals = _mixed_batch(20, 11)
    dg = [to_device(h, dev) for h in graphs]
    plan = _plan(ctx, dg, graphs, ss, duals)
    try:
        for bump in (1, 3, 0):
            s2 = [s + bump for s in ss]
            print(f"case: plan larger s bump={bump}", flush=True)
            _check(plan.run(s2), graphs, s2, duals, f"s + {bump}")
        # below the planned s is refused on the host, and the plan still runs
        from paper_2010_11448_amd import sline

        low = [max(s - 1, 0) for s in ss]
        if any(a < b for a, b in zip(low, ss)):
            assert plan.run_raw(low) == sline.SLINE_EINVAL
        _check(plan.run(), graphs, ss, duals, "after a refused run")
    finally:
        plan.close()


def test_plan_refused_run_changes_no_s(ctx, dev):
    """A run refused for one graph's s changes no graph's s: when an earlier
    graph asked for a larger s in the refused run, the next run that asks
    for that s counts it at that s (and a run at the planned s after that
    counts every graph at its planned s)."""
    from paper_2010_11448_amd import sline

    graphs, ss, duals = _mixed_batch(12, 5)
    dg = [to_device(h, dev) for h in graphs]

    def count(g, s):
        h = graphs[g]
        ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=duals[g],
                              threads=8)
        return len(ref.a)

    # a graph whose L_s changes when its s goes up by two, then a later one
    g0 = next(g for g in range(len(graphs) - 1) if count(g, ss[g]) != count(g, ss[g] + 2))
    g1 = len(graphs) - 1
    plan = _plan(ctx, dg, graphs, ss, duals)
    try:
        bad = list(ss)
        bad[g0] = ss[g0] + 2
        bad[g1] = ss[g1] - 1
        print(f"case: plan refused run s={bad}", flush=True)
        assert plan.run_raw(bad) == sline.SLINE_EINVAL
        good = list(ss)
        good[g0] = ss[g0] + 2
        _check(plan.run(good), graphs, good, duals, "after a refused run")
        _check(plan.run(), graphs, ss, duals, "planned s")
    finally:
        plan.close()


def test_plan_closed_with_its_context(dev):
    """Closing a context destroys its open plans first (a plan belongs to its
    context): closing the plan afterwards does nothing and running it raises.
    A run given the wrong number of s values is refused in the binding."""
    from paper_2010_11448_amd import sline

    graphs, ss, duals = _mixed_batch(4, 2)
    dg = [to_device(h, dev) for h in graphs]
    c = sline.Context(0)
    plan = _plan(c, dg, graphs, ss, duals)
    print("case: plan closed with its context", flush=True)
    _check(plan.run(), graphs, ss, duals, "before the context closes")
    with pytest.raises(ValueError):
        plan.run_raw(ss[:-1])
    c.close()
    assert not plan.plan
    plan.close()
    with pytest.raises(RuntimeError):
        plan.run()


def _relabel_in_place(h, dual, rp, col, seed):
    """Rename the members of every item (vertices of a primal graph, edges of
    a dual one) by a random permutation and write the result into the same
    device arrays: every overlap, hence L_s, stays the same."""
    import torch

    rng = np.random.default_rng(seed)
    if not dual:
        perm = rng.permutation(h.n_vertices).astype(np.int32)
        new_col = np.empty_like(h.col)
        for e in range(h.n_edges):
            lo, hi = h.row_ptr[e], h.row_ptr[e + 1]
            new_col[lo:hi] = np.sort(perm[h.col[lo:hi]])
        new = gen.Hypergraph(h.row_ptr.copy(), new_col, h.n_edges, h.n_vertices, {})
    else:
        order = rng.permutation(h.n_edges)
        rows = [h.col[h.row_ptr[e]:h.row_ptr[e + 1]] for e in order]
        new = gen.from_sets([r.tolist() for r in rows], h.n_vertices)
    assert int(new.row_ptr[-1]) == int(h.row_ptr[-1])
    rp.copy_(torch.as_tensor(new.row_ptr.astype(np.int32)))
    if col.numel():
        col.copy_(torch.as_tensor(new.col.astype(np.int32)))
    return new


def test_plan_rereads_changed_contents(ctx, dev):
    graphs, ss, duals = _mixed_batch(16, 13)
    dg = [to_device(h, dev) for h in graphs]
    plan = _plan(ctx, dg, graphs, ss, duals)
    try:
        new = [_relabel_in_place(h, d, rp, col, 100 + g)
               for g, (h, d, (rp, col)) in enumerate(zip(graphs, duals, dg))]
        print("case: plan after members renamed in place", flush=True)
        res = plan.run()
        _check(res, graphs, ss, duals, "renamed members (same L_s)")
        # the renamed graphs' own oracle gives the same answer
        _check(res, new, ss, duals, "renamed members (their own oracle)")
    finally:
        plan.close()


def test_plan_rejects_malformed_and_outgrown_runs(ctx, dev):
    import torch
    from paper_2010_11448_amd import sline

    disjoint = gen.from_sets([[0, 1], [2, 3], [4, 5], [6, 7]], 8)
    other = gen.uniform_hypergraph(200, 300, 2, 9, seed=5)
    graphs, ss, duals = [disjoint, other], [1, 2], [0, 0]
    dg = [to_device(h, dev) for h in graphs]
    plan = _plan(ctx, dg, graphs, ss, duals)
    rp0, col0 = dg[0]
    try:
        _check(plan.run(copy=True), graphs, ss, duals, "planned")
        # a member out of range
        keep = col0.clone()
        col0[0] = 8
        print("case: plan run with a member out of range", flush=True)
        assert plan.run_raw() == sline.SLINE_EINVAL
        col0.copy_(keep)
        _check(plan.run(), graphs, ss, duals, "restored after a bad member")
        # a member twice in one row
        col0[1] = col0[0]
        print("case: plan run with a row out of order", flush=True)
        assert plan.run_raw() == sline.SLINE_EINVAL
        col0.copy_(keep)
        _check(plan.run(), graphs, ss, duals, "restored after a row out of order")
        # row_ptr[m] changed
        rp_keep = rp0.clone()
        rp0[-1] = rp0[-1] - 1
        print("case: plan run with row_ptr[m] changed", flush=True)
        assert plan.run_raw() == sline.SLINE_EINVAL
        assert "row_ptr" in sline.sline_last_error(ctx.ctx)
        rp0.copy_(rp_keep)
        _check(plan.run(), graphs, ss, duals, "restored after a shape change")
        # the same edges, now all equal: more tasks and pairs than planned
        col0.copy_(torch.tensor([0, 1, 0, 1, 0, 1, 0, 1], dtype=torch.int32))
        print("case: plan run that outgrows the plan", flush=True)
        assert plan.run_raw() == sline.SLINE_ECAPACITY
        assert "make a new plan" in sline.sline_last_error(ctx.ctx)
        col0.copy_(keep)
        _check(plan.run(), graphs, ss, duals, "restored after an outgrown run")
    finally:
        plan.close()


@pytest.mark.parametrize("pool", ["small", "none"])
def test_plan_without_room_to_stage(ctx, dev, pool):
    """A small pool (tasks without room are counted again by the captured fill
    pass) and no pool at all (the fill pass counts every task)."""
    graphs, ss, duals = _mixed_batch(20, 17)
    dg = [to_device(h, dev) for h in graphs]
    base = ctx.tuning()
    ctx.set_tuning(stage_max_bytes={"small": 1 << 20, "none": 0}[pool])
    try:
        plan = _plan(ctx, dg, graphs, ss, duals)
    finally:
        ctx.set_tuning(**base)
    try:
        for r in range(2):
            print(f"case: plan pool={pool} run {r}", flush=True)
            _check(plan.run(), graphs, ss, duals, f"pool={pool} run {r}")
    finally:
        plan.close()


def test_plan_pairs_only_and_edge_cases(ctx, dev):
    import torch
    from paper_2010_11448_amd import sline

    graphs, ss, duals = _mixed_batch(12, 19)
    dg = [to_device(h, dev) for h in graphs]
    plan = _plan(ctx, dg, graphs, ss, duals, flags=sline.SLINE_NO_WEIGHTS)
    try:
        res = plan.run()
        for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
            ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d)
            assert res[g].w is None
            assert np.array_equal(res[g].a.cpu().numpy(), ref.a), f"graph {g}: a"
            assert np.array_equal(res[g].b.cpu().numpy(), ref.b), f"graph {g}: b"
    finally:
        plan.close()
    # no graphs; only empty graphs; flags a plan does not take
    empty = sline.BatchPlan(ctx, [], [])
    assert empty.run() == []
    empty.close()
    erp = torch.zeros(1, dtype=torch.int32, device=dev)
    ecol = torch.zeros(0, dtype=torch.int32, device=dev)
    none = sline.BatchPlan(ctx, [(erp, ecol, 4), (erp, ecol, 0)], [1, 2], [0, 1])
    assert [len(r) for r in none.run()] == [0, 0]
    none.close()
    with pytest.raises(sline.SlineError):
        sline.BatchPlan(ctx, [(dg[0][0], dg[0][1], graphs[0].n_vertices)], [1], [0],
                        flags=sline.SLINE_RELABEL_DESC)


def test_plan_of_law_graphs(ctx, dev):
    """Graphs of the batched-workload law (sizes capped), each with its own s
    and side, replayed twice."""
    items = gen.batch_workload(40, m_cap=20_000)
    graphs = [it.graph for it in items]
    ss = [it.s for it in items]
    duals = [g % 2 for g in range(len(items))]
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: plan law batch s={ss}", flush=True)
    plan = _plan(ctx, dg, graphs, ss, duals)
    try:
        plan.run()
        _check(plan.run(), graphs, ss, duals, "law batch")
    finally:
        plan.close()


@pytest.mark.parametrize("seed", range(6))
def test_plan_randomized(ctx, dev, seed):
    """Random batches (random sets, sizes, sides, per-graph s) replayed at the
    planned s and at random larger s, every graph against the oracle."""
    rng = np.random.default_rng(1000 + seed)
    G = int(rng.integers(1, 12))
    graphs, ss, duals = [], [], []
    for g in range(G):
        m, n = int(rng.integers(0, 120)), int(rng.integers(1, 90))
        p = float(rng.uniform(0.02, 0.4))
        B = rng.random((m, n)) < p
        graphs.append(gen.from_sets([np.flatnonzero(B[i]).tolist() for i in range(m)], n))
        ss.append(int(rng.integers(1, 5)))
        duals.append(int(rng.integers(0, 2)))
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: plan randomized seed={seed} G={G} s={ss} dual={duals}", flush=True)
    plan = _plan(ctx, dg, graphs, ss, duals)
    try:
        _check(plan.run(), graphs, ss, duals, f"seed {seed} planned s")
        for r in range(3):
            s2 = [s + int(rng.integers(0, 4)) for s in ss]
            _check(plan.run(s2), graphs, s2, duals, f"seed {seed} run {r} s={s2}")
    finally:
        plan.close()
