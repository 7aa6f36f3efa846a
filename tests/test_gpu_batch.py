"""Batched builds (many graphs, each with its own s and side) through the C-ABI.

Bar: bit-exact -- every graph's result equals the oracle's on that graph alone
and the plain single-graph build of the same graph.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2010_11448_amd import gen

from helpers import assert_same, to_device

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


def _mixed_batch(n: int, seed: int):
    """Graphs of the batch law (capped sizes) plus planted and random small ones."""
    st = gen.Stream(seed)
    graphs, ss, duals = [], [], []
    for g in range(n):
        kind = g % 4
        if kind == 0:
            item = gen.batch_graph(g, seed=seed, m_cap=1500)
            h, s = item.graph, item.s
        elif kind == 1:
            h = gen.random_small(40 + g, 30 + g, 10, seed + g)
            s = int(st.integers(1, 4, 1)[0])
        elif kind == 2:
            h = gen.uniform_hypergraph(300, 500, 2, 14, seed + g)
            s = int(st.integers(1, 3, 1)[0])
        else:
            h = gen.nested_chain(20, 5, seed=seed + g)
            s = int(st.integers(1, 60, 1)[0])
        graphs.append(h)
        ss.append(s)
        duals.append(int(st.integers(0, 1, 1)[0]))
    return graphs, ss, duals


@pytest.mark.parametrize("seed", [3, 4])
def test_batch_matches_oracle_and_plain(ctx, dev, seed):
    graphs, ss, duals = _mixed_batch(24, seed)
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: batch seed={seed} graphs={len(graphs)} s={ss} dual={duals}", flush=True)
    res = ctx.build_batch([(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)], ss, duals)
    assert len(res) == len(graphs)
    for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
        ref, _ = oracle.naive(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
        assert_same(res[g], ref, f"batch graph {g} s={s} dual={d}")
        rp, col = dg[g]
        alone = ctx.build(rp, col, h.n_vertices, s, d)
        assert_same(alone, ref, f"alone graph {g}")


@pytest.mark.parametrize("pool", ["default", "small", "none"])
def test_batch_library_outputs(ctx, dev, pool):
    """Library-allocated outputs: each graph's pairs are written straight into
    its own arrays, by the staged copy, by the fill pass over tasks the pool
    had no room for ("small"), or by a fill pass over every task ("none")."""
    graphs, ss, duals = _mixed_batch(20, 5)
    dg = [to_device(h, dev) for h in graphs]
    base = ctx.tuning()
    stage = {"default": base["stage_max_bytes"], "small": 1 << 20, "none": 0}[pool]
    print(f"case: batch library outputs pool={pool} s={ss} dual={duals}", flush=True)
    ctx.set_tuning(stage_max_bytes=stage)
    try:
        res = ctx.build_batch([(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)], ss,
                              duals, library_alloc=True)
    finally:
        ctx.set_tuning(**base)
    assert len(res) == len(graphs)
    for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
        ref, _ = oracle.naive(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
        assert_same(res[g], ref, f"library outputs pool={pool} graph {g} s={s} dual={d}")


def test_batch_library_outputs_pairs_only(ctx, dev):
    from paper_2010_11448_amd import sline

    graphs, ss, duals = _mixed_batch(12, 6)
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: batch library outputs pairs only s={ss} dual={duals}", flush=True)
    res = ctx.build_batch([(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)], ss, duals,
                          flags=sline.SLINE_NO_WEIGHTS, library_alloc=True)
    for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
        ref, _ = oracle.naive(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
        assert res[g].w is None
        assert np.array_equal(res[g].a.cpu().numpy(), ref.a), f"graph {g}: a"
        assert np.array_equal(res[g].b.cpu().numpy(), ref.b), f"graph {g}: b"


def test_batch_of_law_graphs_against_wedge_oracle(ctx, dev):
    """Graphs drawn from the batched-workload law (sizes capped) with their own s."""
    items = gen.batch_workload(12, m_cap=20_000)
    graphs = [it.graph for it in items]
    ss = [it.s for it in items]
    duals = [g % 2 for g in range(len(items))]
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: law batch s={ss}", flush=True)
    res = ctx.build_batch([(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)], ss, duals)
    for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
        ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
        assert_same(res[g], ref, f"law graph {g} s={s} dual={d}")


def test_batch_edge_cases(ctx, dev):
    import torch
    from paper_2010_11448_amd import sline

    assert ctx.build_batch([], [], []) == []
    empty_rp = torch.zeros(1, dtype=torch.int32, device=dev)
    empty_col = torch.zeros(0, dtype=torch.int32, device=dev)
    one = gen.from_sets([[0, 1, 2], [1, 2], [2]], 3)
    rp1, col1 = to_device(one, dev)
    res = ctx.build_batch([(empty_rp, empty_col, 4), (rp1, col1, 3), (empty_rp, empty_col, 0)],
                          [1, 1, 2], [0, 1, 1])
    assert [len(r) for r in res] == [0, len(oracle.naive(one.row_ptr, one.col, 3, 3, 1, dual=1)[0]), 0]
    ref, _ = oracle.naive(one.row_ptr, one.col, 3, 3, 1, dual=1)
    assert_same(res[1], ref, "dual in batch with empty graphs")
    # a malformed graph anywhere in the batch fails the whole call
    bad_rp = torch.tensor([0, 2, 4], dtype=torch.int32, device=dev)
    bad_col = torch.tensor([0, 1, 1, 1], dtype=torch.int32, device=dev)
    for d in (0, 1):
        with pytest.raises(sline.SlineError) as ei:
            ctx.build_batch([(rp1, col1, 3), (bad_rp, bad_col, 3)], [1, 1], [0, d])
        assert ei.value.status == sline.SLINE_EINVAL
    with pytest.raises(sline.SlineError) as ei:
        ctx.build_batch([(rp1, col1, 3)], [0], [0])
    assert ei.value.status == sline.SLINE_EINVAL


def test_batch_capacity_protocol(ctx, dev):
    """ECAPACITY reports every graph's size; the retry writes the same result."""
    import torch
    from paper_2010_11448_amd import sline

    graphs = [gen.uniform_2000(11), gen.uniform_2000(12)]
    dg = [to_device(h, dev) for h in graphs]
    csrs = [sline.Context.csr(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)]
    small = torch.zeros(3 * 4, dtype=torch.int32, device=dev)
    outs = (sline.sline_edges * 2)()
    for g in range(2):
        outs[g] = sline.sline_edges(0, 2, small[6 * g:].data_ptr(), small[6 * g + 2:].data_ptr(),
                                    small[6 * g + 4:].data_ptr())
    st = sline.sline_build_batch(ctx.ctx, csrs, [1, 2], [0, 0], 0, outs)
    assert st == sline.SLINE_ECAPACITY
    need = [int(outs[g].n_pairs) for g in range(2)]
    refs = [oracle.naive(h.row_ptr, h.col, h.n_edges, h.n_vertices, s)[0]
            for h, s in zip(graphs, [1, 2])]
    assert need == [len(r) for r in refs]
    bufs = [torch.zeros((3, n), dtype=torch.int32, device=dev) for n in need]
    for g in range(2):
        outs[g] = sline.sline_edges(0, need[g], bufs[g][0].data_ptr(), bufs[g][1].data_ptr(),
                                    bufs[g][2].data_ptr())
    assert sline.sline_build_batch(ctx.ctx, csrs, [1, 2], [0, 0], 0, outs) == sline.SLINE_OK
    for g in range(2):
        assert_same(sline.LineGraph(bufs[g][0], bufs[g][1], bufs[g][2]), refs[g], f"retry graph {g}")
    # library-allocated outputs, freed per graph
    outs = (sline.sline_edges * 2)()
    assert sline.sline_build_batch(ctx.ctx, csrs, [1, 2], [0, 0], 0, outs) == sline.SLINE_OK
    assert [int(outs[g].n_pairs) for g in range(2)] == need
    for g in range(2):
        assert sline.sline_edges_free(ctx.ctx, outs[g]) == sline.SLINE_OK


def test_full_lognormal_batch_every_graph(ctx, dev):
    """The batched workload at its stated size -- 512 graphs, m_g lognormal on
    [1e3, 2e5], each with its own s on 1..12 -- in the launch configuration the
    bench times (one sline_build_batch, library-allocated results): every
    graph's result equals O3 on that graph alone, element by element."""
    import os
    import time

    import torch

    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.time()
    items = gen.batch_workload(512)
    print(f"case: full lognormal batch of {len(items)} graphs "
          f"(generated in {time.time() - t0:.1f} s)", flush=True)
    dg = [to_device(it.graph, dev) for it in items]
    ss = [it.s for it in items]
    duals = [it.dual for it in items]
    res = ctx.build_batch([(rp, col, it.graph.n_vertices) for (rp, col), it in zip(dg, items)],
                          ss, duals, library_alloc=True)
    del dg
    t1 = time.time()
    total = 0
    for g, (it, L) in enumerate(zip(items, res)):
        h = it.graph
        ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, it.s, dual=it.dual,
                              threads=threads)
        assert_same(L, ref, f"lognormal batch graph {g} (m={h.n_edges}) s={it.s} dual={it.dual}")
        total += len(L)
        res[g] = None
    print(f"case: full lognormal batch: {total} pairs checked in {time.time() - t1:.1f} s",
          flush=True)
    torch.cuda.empty_cache()


def test_batch_with_cached_tuning(ctx, dev, tmp_path):
    """An autotuner cache entry for the batch's class applies to the batched
    call and to a plan made from it (same results), and the context's own
    tuning is back afterwards."""
    from paper_2010_11448_amd import autotune, sline

    graphs, ss, duals = _mixed_batch(16, 23)
    dg = [to_device(h, dev) for h in graphs]
    tg = [(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)]
    path = str(tmp_path / "tune.json")
    entry = {"small_slots": 2048, "small_max_wedges": 1024, "task_slots": 13440,
             "task_grid_per_cu": 2, "task_wedges": 3500}
    autotune.save_cached(path, autotune.batch_signature(tg, ss, duals), entry, 0.1)
    before = ctx.tuning()
    print("case: batch with a cached tuning", flush=True)
    res = ctx.build_batch(tg, ss, duals, tuning_cache=path)
    assert ctx.tuning() == before
    plan = sline.BatchPlan(ctx, tg, ss, duals, tuning_cache=path)
    assert ctx.tuning() == before
    try:
        pres = plan.run()
        for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
            ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
            assert_same(res[g], ref, f"cached tuning graph {g}")
            assert_same(pres[g], ref, f"cached tuning plan graph {g}")
    finally:
        plan.close()
