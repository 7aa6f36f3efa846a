"""Serving (continuous batching) through the C-ABI.

Bar: bit-exact -- every query answered by the server, whatever batch it ran
in, equals the plain build of the same graph, s and side (and the oracle).
"""

from __future__ import annotations

import time

import pytest

import oracle
from paper_2010_11448_amd import gen

from helpers import assert_same, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available()
    return torch.device("cuda", 0)


def _catalog():
    graphs = [gen.uniform_2000(11), gen.uniform_2000(12), gen.powerlaw_1m(scale=0.01),
              gen.random_small(60, 40, 12, 7), gen.sunflower(300, 6, 5, seed=3),
              gen.nested_chain(40, 7, seed=4)]
    graphs += [gen.batch_graph(g, m_cap=3000).graph for g in range(6)]
    return graphs


def _drain(srv, tickets, timeout_s=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t in done:
                continue
            r = srv.poll(t)
            if r is not None:
                done[t] = r
        assert time.time() - t0 < timeout_s, "server did not finish"
        time.sleep(0.001)
    return done


@pytest.mark.parametrize("workers,budget,reuse", [(2, 64 << 30, False), (1, 1 << 20, False),
                                                  (2, 64 << 30, True), (3, 8 << 30, True),
                                                  (3, 64 << 30, "lookahead")])
def test_mixed_queries_equal_alone(dev, workers, budget, reuse):
    from paper_2010_11448_amd import sline

    graphs = _catalog()
    dg = [to_device(h, dev) for h in graphs]
    srv = sline.Server(0, hbm_budget_bytes=budget, max_batch=16, workers=workers)
    # reuse on every graph (kept results answer later queries by a filter),
    # with queued queries of one graph and side built once at their smallest
    # s (lookahead), or none at all
    srv.set_reuse(1 << 30 if reuse else 0, 0, lookahead=reuse == "lookahead")
    ctx = sline.Context(0)
    try:
        ids = [srv.register(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)]
        st = gen.Stream(99)
        queries = []
        for _ in range(60):
            g = int(st.integers(0, len(graphs) - 1, 1)[0])
            queries.append((g, int(st.integers(1, 6, 1)[0]), int(st.integers(0, 1, 1)[0])))
        print(f"case: serve workers={workers} budget={budget} queries={len(queries)}", flush=True)
        tickets = [srv.submit(ids[g], s, d) for g, s, d in queries]
        done = _drain(srv, tickets)
        sizes = [done[t][1]["batch_size"] for t in tickets]
        if budget >= 1 << 30 and not reuse:
            assert max(sizes) > 1, "queries submitted together should share batches"
        elif budget < 1 << 30:
            # every estimate exceeds a 1 MiB budget: each query runs alone
            assert max(sizes) == 1
        if reuse:
            assert srv.reuse_stats()["reused"] > 0, "no query was answered from a kept result"
        else:
            assert srv.reuse_stats()["reused"] == 0
        for (g, s, d), t in zip(queries, tickets):
            L, info = done[t]
            assert info["status"] == 0 and info["n_pairs"] == len(L)
            assert info["t_submit_ns"] <= info["t_start_ns"] <= info["t_done_ns"]
            rp, col = dg[g]
            alone = ctx.build(rp, col, graphs[g].n_vertices, s, d)
            assert_same(L, oracle.Pairs(alone.a.cpu().numpy(), alone.b.cpu().numpy(),
                                        alone.w.cpu().numpy()),
                        f"graph {g} s={s} dual={d} in a batch of {info['batch_size']}")
        # one query per graph against the oracle as well
        for g in range(len(graphs)):
            h = graphs[g]
            ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, 2, dual=g % 2,
                                  threads=8)
            t = srv.submit(ids[g], 2, g % 2)
            L, _ = _drain(srv, [t])[t]
            assert_same(L, ref, f"served graph {g} vs oracle")
    finally:
        srv.close()
        ctx.close()


def test_unreleased_results_do_not_stall(dev):
    """Results the client leaves unreleased count against the budget; with the
    budget full of them, a query still runs when nothing else does, so every
    query finishes although nothing is polled until the end."""
    from paper_2010_11448_amd import sline

    graphs = [gen.uniform_2000(11), gen.uniform_2000(12), gen.random_small(60, 40, 12, 7)]
    dg = [to_device(h, dev) for h in graphs]
    srv = sline.Server(0, hbm_budget_bytes=1 << 22, max_batch=8, workers=2)
    ctx = sline.Context(0)
    try:
        ids = [srv.register(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)]
        queries = [(g % 3, 1 + g % 4, g % 2) for g in range(24)]
        print(f"case: serve unreleased results queries={len(queries)}", flush=True)
        tickets = [srv.submit(ids[g], s, d) for g, s, d in queries]
        t0 = time.time()
        while srv.pending() != (0, 0):
            assert time.time() - t0 < 120, "server stalled with unreleased results"
            time.sleep(0.005)
        for (g, s, d), t in reversed(list(zip(queries, tickets))):
            L, info = srv.poll(t)
            assert info["status"] == 0
            rp, col = dg[g]
            alone = ctx.build(rp, col, graphs[g].n_vertices, s, d)
            assert_same(L, oracle.Pairs(alone.a.cpu().numpy(), alone.b.cpu().numpy(),
                                        alone.w.cpu().numpy()), f"graph {g} s={s} dual={d}")
    finally:
        srv.close()
        ctx.close()


def test_server_errors(dev):
    from paper_2010_11448_amd import sline

    srv = sline.Server(0, hbm_budget_bytes=1 << 30, max_batch=4, workers=1)
    try:
        g = gen.uniform_2000(11)
        rp, col = to_device(g, dev)
        gid = srv.register(rp, col, g.n_vertices)
        for bad in ((gid, 0, 0), (gid, 1, 2), (gid + 5, 1, 0)):
            with pytest.raises(sline.SlineError) as ei:
                srv.submit(*bad)
            assert ei.value.status == sline.SLINE_EINVAL
        with pytest.raises(sline.SlineError):
            srv.poll(12345)
        t = srv.submit(gid, 3, 0)
        L, info = _drain(srv, [t])[t]
        assert info["n_pairs"] == len(L)
        assert srv.pending() == (0, 0)
    finally:
        srv.close()


def test_malformed_graphs_refused_at_registration(dev):
    """A graph that breaks the CSR rules is refused when it is registered, so
    it can never join (and fail) a batch; valid queries submitted afterwards
    still equal their plain builds."""
    import numpy as np
    import torch
    from paper_2010_11448_amd import sline

    good = gen.uniform_2000(13)
    bad_sets = {
        "row_ptr[0] != 0": (np.array([1, 3, 5], np.int32), np.array([0, 1, 2, 3, 4], np.int32)),
        "unsorted row": (np.array([0, 3, 5], np.int32), np.array([2, 1, 3, 0, 4], np.int32)),
        "repeated member": (np.array([0, 3, 5], np.int32), np.array([1, 1, 3, 0, 4], np.int32)),
        "member out of range": (np.array([0, 2, 4], np.int32), np.array([0, 9, 1, 2], np.int32)),
        "row_ptr decreases": (np.array([0, 4, 2, 5], np.int32),
                              np.array([0, 1, 2, 3, 4], np.int32)),
    }
    srv = sline.Server(0, hbm_budget_bytes=1 << 30, max_batch=16, workers=2)
    ctx = sline.Context(0)
    try:
        rp, col = to_device(good, dev)
        gid = srv.register(rp, col, good.n_vertices)
        keep = []
        for what, (brp, bcol) in bad_sets.items():
            print(f"case: serve register refuses {what}", flush=True)
            drp = torch.from_numpy(brp).to(dev)
            dcol = torch.from_numpy(bcol).to(dev)
            keep.append((drp, dcol))
            with pytest.raises(sline.SlineError) as ei:
                srv.register(drp, dcol, 5)
            assert ei.value.status == sline.SLINE_EINVAL, what
        tickets = [(srv.submit(gid, s_, d_), s_, d_) for s_ in (1, 2, 3) for d_ in (0, 1)]
        done = _drain(srv, [t for t, _, _ in tickets])
        for t, s_, d_ in tickets:
            L, info = done[t]
            assert info["status"] == 0
            alone = ctx.build(rp, col, good.n_vertices, s_, d_)
            assert_same(L, oracle.Pairs(alone.a.cpu().numpy(), alone.b.cpu().numpy(),
                                        alone.w.cpu().numpy()), f"s={s_} dual={d_}")
    finally:
        srv.close()
        ctx.close()


def test_fullsize_queries_in_the_mix(dev):
    """Queries on the 1,000,000 x 2,000,000 power-law graph (s = 2 and 16, both
    sides) submitted together with small queries: each served result equals
    the plain build of the same query, compared element by element on the
    device (the plain build itself is checked against the oracle at this size
    in test_gpu_fullsize.py)."""
    import torch
    from paper_2010_11448_amd import sline

    big = gen.powerlaw_1m()
    small = [gen.uniform_2000(11), gen.batch_graph(3).graph, gen.batch_graph(9).graph]
    dbig = to_device(big, dev)
    dsmall = [to_device(h, dev) for h in small]
    srv = sline.Server(0, hbm_budget_bytes=96 << 30, max_batch=16, workers=3)
    ctx = sline.Context(0)
    try:
        gbig = srv.register(dbig[0], dbig[1], big.n_vertices)
        gsm = [srv.register(rp, col, h.n_vertices) for (rp, col), h in zip(dsmall, small)]
        queries = []
        for s_, d_ in ((2, 0), (16, 0), (2, 1), (16, 1)):
            queries.append((None, s_, d_))
            for i in range(len(small)):
                queries.append((i, 1 + (s_ + i) % 5, (d_ + i) % 2))
        print(f"case: serve full-size power-law queries in a mix of {len(queries)}", flush=True)
        tickets = [srv.submit(gbig if g is None else gsm[g], s_, d_) for g, s_, d_ in queries]
        done = _drain(srv, tickets, timeout_s=300.0)
        for (g, s_, d_), t in zip(queries, tickets):
            L, info = done[t]
            assert info["status"] == 0
            if g is None:
                rp, col, nv, what = dbig[0], dbig[1], big.n_vertices, f"full size s={s_} dual={d_}"
            else:
                (rp, col), nv = dsmall[g], small[g].n_vertices
                what = f"small graph {g} s={s_} dual={d_}"
            alone = ctx.build(rp, col, nv, s_, d_)
            assert len(L) == len(alone), what
            for x, y, name in ((L.a, alone.a, "a"), (L.b, alone.b, "b"), (L.w, alone.w, "w")):
                assert torch.equal(x, y), f"{what}: {name} differs from the plain build"
            del L, alone
            done[t] = None
            torch.cuda.empty_cache()
    finally:
        srv.close()
        ctx.close()
