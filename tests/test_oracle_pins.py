"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test ties O1 (the definition evaluated pair by pair) or O3 (wedge counting
with exact counters) to something independent: a library routine (dense BLAS
product B B^T in float64, exact for these counts; networkx line graphs), closed
forms, structural special cases, brute-force invariants, and the worked
example of Sec. I / Sec. IV (the sets its text fixes).
"""

from __future__ import annotations

import itertools
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2010_11448_amd import gen

from helpers import digest_torch, mix_py

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pairs_from_dense(Wm: np.ndarray, s: int):
    """(a, b, w) with a < b and W[a, b] >= s, in (a, b) order, from a dense overlap matrix."""
    iu = np.triu_indices(Wm.shape[0], k=1)
    w = Wm[iu]
    keep = w >= s
    return iu[0][keep].astype(np.int32), iu[1][keep].astype(np.int32), w[keep].astype(np.int32)


def incidence(g) -> np.ndarray:
    """Dense hyperedge x vertex 0/1 matrix (float64) built with numpy only."""
    B = np.zeros((g.n_edges, g.n_vertices), dtype=np.float64)
    rows = np.repeat(np.arange(g.n_edges), np.diff(g.row_ptr))
    B[rows, g.col] = 1.0
    return B


def check_against_dense(g, s, dual):
    B = incidence(g)
    Wm = (B.T @ B) if dual else (B @ B.T)
    a, b, w = pairs_from_dense(np.rint(Wm).astype(np.int64), s)
    got, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=4)
    assert np.array_equal(got.a, a) and np.array_equal(got.b, b) and np.array_equal(got.w, w)


def csr_from_dense(B: np.ndarray):
    rp = np.zeros(B.shape[0] + 1, dtype=np.int32)
    rp[1:] = np.cumsum(B.sum(axis=1))
    col = np.nonzero(B)[1].astype(np.int32)
    return gen.Hypergraph(rp, col, B.shape[0], B.shape[1], {})


# ----------------------------------------------------- library routine

@settings(max_examples=60, deadline=None)
@given(st.integers(0, 30), st.integers(1, 30), st.floats(0.0, 0.6), st.integers(0, 2**31 - 1),
       st.integers(1, 5))
def test_o1_equals_blas_product_on_tiny_graphs(m, n, p, seed, s):
    rng = np.random.default_rng(seed)
    B = (rng.random((m, n)) < p).astype(np.int64)
    g = csr_from_dense(B)
    for dual in (0, 1):
        check_against_dense(g, s, dual)


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 30), st.integers(1, 30), st.floats(0.0, 0.6), st.integers(0, 2**31 - 1),
       st.integers(1, 5), st.integers(1, 4))
def test_o3_equals_blas_product_on_tiny_graphs(m, n, p, seed, s, threads):
    """O3 pinned to the dense product directly, not through O1."""
    rng = np.random.default_rng(seed)
    B = (rng.random((m, n)) < p).astype(np.int64)
    g = csr_from_dense(B)
    for dual in (0, 1):
        Wm = (B.T @ B) if dual else (B @ B.T)
        a, b, w = pairs_from_dense(Wm, s)
        got, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                              threads=threads)
        assert np.array_equal(got.a, a) and np.array_equal(got.b, b) and np.array_equal(got.w, w)


@pytest.mark.parametrize("seed", gen.UNIFORM_SEEDS)
def test_o1_equals_blas_product_on_uniform_2000(seed):
    g = gen.uniform_2000(seed)
    for s in gen.UNIFORM_S:
        check_against_dense(g, s, 0)
    for s in (1, 2, 3):
        check_against_dense(g, s, 1)


# -------------------------------------------------------- special cases

def test_l1_of_a_graph_is_the_networkx_line_graph():
    nx = pytest.importorskip("networkx")
    st_ = gen.Stream(5)
    n = 60
    edges = set()
    while len(edges) < 150:
        u, v = st_.integers(0, n - 1, 2)
        if u != v:
            edges.add((min(int(u), int(v)), max(int(u), int(v))))
    edges = sorted(edges)
    g = gen.from_sets([list(e) for e in edges], n)
    got, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    G = nx.Graph()
    G.add_edges_from(edges)
    LG = nx.line_graph(G)
    idx = {e: i for i, e in enumerate(edges)}
    want = sorted(tuple(sorted((idx[tuple(sorted(x))], idx[tuple(sorted(y))]))) for x, y in LG.edges())
    assert list(zip(got.a.tolist(), got.b.tolist())) == want
    assert (got.w == 1).all()
    # parallel copies of an edge overlap in both endpoints
    g2 = gen.from_sets([list(e) for e in edges] + [list(edges[0])], n)
    got2, _ = oracle.naive(g2.row_ptr, g2.col, g2.n_edges, g2.n_vertices, 2)
    assert list(zip(got2.a.tolist(), got2.b.tolist(), got2.w.tolist())) == [(0, len(edges), 2)]


def test_weight_sum_closed_form():
    for g in (gen.uniform_2000(11), gen.random_small(80, 50, 15, 3), gen.powerlaw_1m(scale=0.005)):
        deg = np.bincount(g.col, minlength=g.n_vertices).astype(np.int64)
        size = np.diff(g.row_ptr).astype(np.int64)
        _, st1 = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1, keep=False)
        assert st1.sum_w == int((deg * (deg - 1) // 2).sum())
        _, st2 = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1, dual=1, keep=False)
        assert st2.sum_w == int((size * (size - 1) // 2).sum())


def test_structure_families():
    # pairwise disjoint hyperedges: empty line graph
    g = gen.from_sets([[3 * i, 3 * i + 1, 3 * i + 2] for i in range(20)], 60)
    assert len(oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)[0]) == 0
    # sunflower: every pair overlaps in exactly the core
    g = gen.sunflower(25, 4, 3, seed=2)
    p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    assert len(p) == 25 * 24 // 2 and (p.w == 4).all()
    assert len(oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 5)[0]) == 0
    # every hyperedge is the whole vertex set
    g = gen.from_sets([list(range(9))] * 7, 9)
    p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 9)
    assert len(p) == 21 and (p.w == 9).all()
    # nested chain: overlap is the smaller set
    g = gen.nested_chain(15, 4, seed=1)
    size = np.diff(g.row_ptr)
    p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    assert len(p) == 15 * 14 // 2
    assert (p.w == np.minimum(size[p.a], size[p.b])).all()


def test_worked_example_text_facts():
    spec = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    names = ["A", "B", "C", "D"]
    sets = [[v - 1 for v in spec["completion"][k]] for k in names]
    fixed = spec["text_fixed"]
    assert spec["completion"]["B"] == fixed["B"]
    g = gen.from_sets(sets, fixed["n_vertices"])
    size = np.diff(g.row_ptr)
    for k, v in fixed["sizes"].items():
        assert size[names.index(k)] == v
    w = {}
    for s in range(1, 5):
        p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s)
        got = [[names[a], names[b], int(x)] for a, b, x in zip(p.a, p.b, p.w)]
        assert got == spec["completion_line_graphs"][str(s)]
        if s == 1:
            w = {names[a] + names[b]: int(x) for a, b, x in zip(p.a, p.b, p.w)}
    for pair, val in fixed["overlaps"].items():
        assert w.get(pair, 0) == val
    # in the dual, vertices 8, 9, 10 lie in both B and C: they overlap in 2 items
    p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 2, dual=1)
    got = {(int(a), int(b)): int(x) for a, b, x in zip(p.a, p.b, p.w)}
    for u, v in itertools.combinations([8, 9, 10], 2):
        assert got[(u - 1, v - 1)] == 2


# ------------------------------------------------------------ invariants

def test_monotone_in_s_and_filter_of_l1():
    g = gen.powerlaw_1m(scale=0.003)
    p1, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1, threads=8)
    prev = p1.as_set()
    for s in range(2, 8):
        ps, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, threads=8)
        cur = ps.as_set()
        assert cur <= prev
        keep = p1.w >= s
        assert np.array_equal(ps.a, p1.a[keep]) and np.array_equal(ps.w, p1.w[keep])
        prev = cur


def test_pruning_and_bounds():
    g = gen.random_small(70, 30, 14, seed=8)
    size = np.diff(g.row_ptr)
    for s in range(1, 8):
        p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s)
        assert (size[p.a] >= s).all() and (size[p.b] >= s).all()
        assert (p.w <= np.minimum(size[p.a], size[p.b])).all()
        assert (p.a < p.b).all()
        q, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, skip_small=True)
        assert p.as_set() == q.as_set()


def test_symmetric_by_brute_force():
    g = gen.random_small(25, 12, 8, seed=4)
    rows = [set(g.col[g.row_ptr[i]:g.row_ptr[i + 1]].tolist()) for i in range(g.n_edges)]
    p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    got = {(a, b): w for a, b, w in zip(p.a.tolist(), p.b.tolist(), p.w.tolist())}
    for a in range(g.n_edges):
        for b in range(g.n_edges):
            if a == b:
                continue
            w = len(rows[a] & rows[b])
            key = (min(a, b), max(a, b))
            assert got.get(key, 0) == w


def test_dual_is_the_transposed_hypergraph():
    sp = pytest.importorskip("scipy.sparse")
    g = gen.random_small(50, 35, 10, seed=6)
    B = sp.csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n_edges, g.n_vertices))
    T = B.T.tocsr()
    T.sort_indices()
    gt = gen.Hypergraph(T.indptr.astype(np.int32), T.indices.astype(np.int32), g.n_vertices,
                        g.n_edges, {})
    for s in (1, 2, 3):
        d, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=1)
        t, _ = oracle.naive(gt.row_ptr, gt.col, gt.n_edges, gt.n_vertices, s)
        assert d.as_set() == t.as_set()
        # (H*)* = H
        dd, _ = oracle.naive(gt.row_ptr, gt.col, gt.n_edges, gt.n_vertices, s, dual=1)
        pp, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s)
        assert dd.as_set() == pp.as_set()
    rpT, colT = oracle.transpose(g.row_ptr, g.col, g.n_edges, g.n_vertices)
    assert np.array_equal(rpT, gt.row_ptr) and np.array_equal(colT, gt.col)


def test_relabel_permutes_the_output():
    g = gen.uniform_hypergraph(300, 200, 2, 12, seed=3)
    perm = np.argsort(gen.Stream(4).uniform(g.n_edges), kind="stable")  # new id -> old id
    rows = [g.col[g.row_ptr[i]:g.row_ptr[i + 1]].tolist() for i in perm]
    h = gen.from_sets(rows, g.n_vertices)
    old_of_new = perm
    for s in (1, 2, 3):
        p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s)
        q, _ = oracle.naive(h.row_ptr, h.col, h.n_edges, h.n_vertices, s)
        mapped = {(min(old_of_new[a], old_of_new[b]), max(old_of_new[a], old_of_new[b]), w)
                  for a, b, w in zip(q.a.tolist(), q.b.tolist(), q.w.tolist())}
        assert mapped == p.as_set()


def test_naive_makes_all_pairs_intersections():
    for m in (0, 1, 2, 37, 500):
        g = gen.uniform_hypergraph(m, 50, 1, 5, seed=m + 1)
        _, st_ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1, keep=False)
        assert st_.intersections == m * (m - 1) // 2
    # Table I lists 3.52e10 naive intersections for 265.2k hyperedges: m(m-1)/2
    m = 265_200
    assert abs(m * (m - 1) / 2 - 3.52e10) / 3.52e10 < 0.005


def test_results_do_not_depend_on_thread_count():
    g = gen.powerlaw_1m(scale=0.002)
    base, bst = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 2, threads=1)
    for t in (3, 8):
        p, pst = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 2, threads=t)
        assert np.array_equal(p.a, base.a) and np.array_equal(p.b, base.b) and np.array_equal(p.w, base.w)
        assert pst.digest == bst.digest


# ----------------------------------------------------------- O3 vs O1

def _same(p, q):
    return np.array_equal(p.a, q.a) and np.array_equal(p.b, q.b) and np.array_equal(p.w, q.w)


@pytest.mark.parametrize("seed", gen.UNIFORM_SEEDS)
def test_o3_equals_o1_uniform_2000(seed):
    g = gen.uniform_2000(seed)
    for dual in (0, 1):
        for s in gen.UNIFORM_S:
            p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
            q, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
            assert _same(p, q)


def test_o3_equals_o1_on_planted_and_random():
    cases = [gen.sunflower(40, 5, 4, 1), gen.nested_chain(30, 5, 2),
             gen.planted_copies(gen.uniform_hypergraph(60, 80, 3, 9, 5), 3, 6)]
    cases += [gen.random_small(90, 40, 15, sd) for sd in range(5)]
    for g in cases:
        for dual in (0, 1):
            for s in (1, 2, 3, 5, 9):
                p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual)
                q, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual)
                assert _same(p, q)


def test_o3_equals_o1_on_scaled_powerlaw():
    g = gen.powerlaw_1m(scale=0.01)  # 10k hyperedges, 20k vertices
    for dual, ss in ((0, (1, 2, 4, 8, 16)), (1, (2, 8, 32))):
        for s in ss:
            p, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                skip_small=True, threads=8)
            q, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
            assert _same(p, q)


def test_o3_wedge_count_closed_form():
    g = gen.powerlaw_1m(scale=0.01)
    size = np.diff(g.row_ptr).astype(np.int64)
    for s in (1, 2, 4, 8):
        kept = size >= s
        rows = np.repeat(np.arange(g.n_edges), size)
        d_s = np.bincount(g.col[kept[rows]], minlength=g.n_vertices).astype(np.int64)
        _, st_ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, keep=False)
        assert st_.wedges == int((d_s * (d_s - 1) // 2).sum())


# --------------------------------------------------------------- digests

def test_digest_terms_and_sum():
    for a, b, w in [(0, 1, 1), (5, 7, 3), (2**31 - 2, 2**31 - 1, 9999), (123456, 654321, 17)]:
        assert oracle.mix(a, b, w) == mix_py(a, b, w)
    g = gen.uniform_2000(13)
    p, st_ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    want = sum(mix_py(int(a), int(b), int(w)) for a, b, w in zip(p.a, p.b, p.w)) % (1 << 64)
    assert st_.digest == want
    import torch
    assert digest_torch(torch.from_numpy(p.a), torch.from_numpy(p.b), torch.from_numpy(p.w),
                        chunk=7777) == want
