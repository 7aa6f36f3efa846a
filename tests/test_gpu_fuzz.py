"""Seeded shapes at the path's internal boundaries, against the oracle.

The counting path changes its course at fixed sizes: an item's wedge cost
W_a decides between the one-wave kernel and the workgroup tasks, tasks hold
a fixed number of wedges, a member list is walked by one lane or in pieces of
whole waves, a workgroup's table holds a fixed number of keys before the key
range is split, and at most s - 1 (capped) member lists are lookup-only.
"Star" hypergraphs put one item's W_a, its number of distinct candidates and
its member-list lengths just below, at and just above each of these sizes,
on both sides.  Random small graphs with a mix of empty, short and long rows
and random s fill in between.  Bar: bit-exact, as every parity test.
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


def star(T: int, k: int, r: int, before: int, after: int, seed: int):
    """A hub item with k members and T later items, each holding r consecutive
    hub members (cyclically) and two private vertices; `before` earlier items
    hold random hub members too, and `after` trailing items hold only private
    vertices.  The hub's wedge cost is r * T over T distinct candidates, each
    with overlap r; a hub member lies in about r * T / k later items.  The
    trailing items crowd the candidates into the first part of the id range
    after the hub, so one of its equal-width tasks gets them all."""
    rng = np.random.default_rng(seed)
    hub = list(range(k))
    nxt = k
    sets = []
    for _ in range(before):
        sets.append(sorted(rng.choice(k, size=min(k, 3), replace=False).tolist() + [nxt]))
        nxt += 1
    sets.append(hub)
    for j in range(T):
        mem = {(j + q) % k for q in range(r)}
        sets.append(sorted(mem) + [nxt, nxt + 1])
        nxt += 2
    for _ in range(after):
        sets.append([nxt, nxt + 1])
        nxt += 2
    return gen.from_sets(sets, nxt)


# (T, k, r): wedge cost r*T around the one-wave limit (512), the task size
# (5000) and its multiples; distinct candidates T around a workgroup table
# (8960 keys); member lists around the 256-entry piece and four pieces.
STARS = [
    (511, 8, 1), (512, 8, 1), (513, 8, 1),
    (256, 2, 2), (257, 2, 2),
    (4999, 20, 1), (5000, 20, 1), (5001, 20, 1), (10001, 40, 1),
    (8959, 35, 1), (8960, 35, 1), (8961, 35, 1), (17921, 70, 2),
    (1023, 1, 1), (1024, 1, 1), (1025, 1, 1), (4100, 4, 1),
    (3000, 40, 17),
]


@pytest.mark.parametrize("T,k,r", STARS, ids=[f"T{t}_k{k}_r{r}" for t, k, r in STARS])
@pytest.mark.parametrize("crowd", [0, 1])
def test_star_boundaries(ctx, dev, T, k, r, crowd):
    g = star(T, k, r, before=5, after=4 * T * crowd, seed=T + k + r)
    rp, col = to_device(g, dev)
    for dual in (0, 1):
        for s in sorted({1, 2, max(1, r - 1), r, r + 1, 16, 17}):
            what = f"star T={T} k={k} r={r} crowd={crowd} s={s} dual={dual}"
            print(f"case: {what}", flush=True)
            L = ctx.build(rp, col, g.n_vertices, s, dual)
            ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                  threads=8)
            assert_same(L, ref, what)


def mixed_rows(seed: int):
    """Random graph whose row lengths mix empty, short and a few long rows."""
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(0, 400))
    n = int(rng.integers(1, 300))
    sets = []
    for _ in range(m):
        u = rng.random()
        if u < 0.1:
            size = 0
        elif u < 0.8:
            size = int(rng.integers(1, 6))
        else:
            size = int(rng.integers(min(6, n), n + 1))
        sets.append(sorted(rng.choice(n, size=min(size, n), replace=False).tolist()))
    return gen.from_sets(sets, n)


@pytest.mark.parametrize("seed", range(40))
def test_mixed_rows_random_s(ctx, dev, seed):
    g = mixed_rows(seed)
    rng = np.random.default_rng(seed)
    rp, col = to_device(g, dev)
    for _ in range(3):
        s = int(rng.integers(1, 21))
        dual = int(rng.integers(0, 2))
        print(f"case: mixed seed={seed} m={g.n_edges} n={g.n_vertices} s={s} dual={dual}",
              flush=True)
        L = ctx.build(rp, col, g.n_vertices, s, dual)
        ref, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                              threads=8)
        assert_same(L, ref, f"mixed seed={seed} s={s} dual={dual}")


@pytest.mark.parametrize("seed", [0, 1])
def test_batch_of_boundary_shapes(ctx, dev, seed):
    """The same shapes in one batch, each graph with its own s and side: the
    per-graph candidate bound and s must hold inside shared tasks."""
    rng = np.random.default_rng(500 + seed)
    graphs, ss, duals = [], [], []
    for i, (T, k, r) in enumerate(STARS):
        graphs.append(star(T, k, r, before=5, after=4 * T * ((i + seed) % 2), seed=T + k + r))
        ss.append(int(rng.choice([1, 2, r, r + 1, 16, 17])))
        duals.append(int(rng.integers(0, 2)))
        graphs.append(mixed_rows(100 + 20 * seed + i))
        ss.append(int(rng.integers(1, 21)))
        duals.append(int(rng.integers(0, 2)))
    dg = [to_device(h, dev) for h in graphs]
    print(f"case: boundary batch seed={seed} graphs={len(graphs)} s={ss} dual={duals}",
          flush=True)
    res = ctx.build_batch([(rp, col, h.n_vertices) for (rp, col), h in zip(dg, graphs)], ss,
                          duals)
    assert len(res) == len(graphs)
    for g, (h, s, d) in enumerate(zip(graphs, ss, duals)):
        ref, _ = oracle.wedge(h.row_ptr, h.col, h.n_edges, h.n_vertices, s, dual=d, threads=8)
        assert_same(res[g], ref, f"boundary batch graph {g} s={s} dual={d}")
