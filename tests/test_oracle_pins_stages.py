"""Pins of the oracle's later-stage functions against facts that do not come
from the oracle itself.

* O2 (the heuristic algorithm of Sec. IV-C with each heuristic a switch, the
  variants f0..f4 of Table III): every variant returns L_s exactly as the
  dense product B B^T says (Sec. V-C: the variants differ in work, not in
  result), and the set intersections each variant makes equal closed forms:
  one per wedge without visited-skipping (sum over members of C(d, 2), with d
  counting only items of size >= s when pruning), one per distinct pair of
  items sharing a member with it (the nonzeros of B B^T above the diagonal).
* filter_s: L_s obtained from a weighted L_1 equals L_s computed directly
  (Sec. III: L_s is L_1 restricted to w >= s).
* squeeze / adjacency (Sec. IV-E): the symmetric adjacency over the squeezed
  ids equals scipy's sparse matrix of the pairs, rows and columns of absent
  items removed.
* components (Table I): the partition equals scipy's connected_components;
  closed forms on planted families.
* relabel (Sec. IV-F): a permutation ordering the sizes, ties by id, after
  which L_s mapped back equals L_s of the original (brute force, O1).
"""

from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2010_11448_amd import gen

from test_oracle_pins import check_against_dense, csr_from_dense, incidence, pairs_from_dense


def _graphs():
    yield gen.random_small(40, 30, 9, seed=1)
    yield gen.random_small(25, 60, 14, seed=2)
    yield gen.uniform_hypergraph(120, 90, 2, 9, seed=3)
    yield gen.sunflower(12, 4, 3, seed=4)
    yield gen.planted_copies(gen.uniform_hypergraph(15, 20, 2, 6, seed=5), 3, seed=6)
    yield gen.nested_chain(10, 3, seed=7)


def _same(P, a, b, w):
    return np.array_equal(P.a, a) and np.array_equal(P.b, b) and np.array_equal(P.w, w)


def _side(g, dual):
    """Dense 0/1 incidence with rows = the side's items."""
    B = incidence(g)
    return B.T if dual else B


# ------------------------------------------------------------------ O2

@pytest.mark.parametrize("variant", sorted(oracle.VARIANTS))
def test_o2_variants_return_the_dense_product_result(variant):
    for g in _graphs():
        for dual in (0, 1):
            B = _side(g, dual)
            Wm = np.rint(B @ B.T).astype(np.int64)
            for s in (1, 2, 3, 5):
                a, b, w = pairs_from_dense(Wm, s)
                got, _ = oracle.alg_h(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                      variant=oracle.VARIANTS[variant], threads=3)
                assert _same(got, a, b, w), (variant, s, dual)


def _intersections_closed_form(B, s, prune, visited):
    """Set intersections the heuristic algorithm makes, from B alone."""
    size = B.sum(axis=1)
    keep = size >= s if prune else np.ones(B.shape[0], dtype=bool)
    Bk = B[keep]
    if visited:
        # one per pair a < b of kept items sharing a member
        Wk = np.rint(Bk @ Bk.T)
        return int(np.count_nonzero(np.triu(Wk, k=1)))
    # one per wedge (a, v, b), a < b, both kept
    d = Bk.sum(axis=0).astype(np.int64)
    return int((d * (d - 1) // 2).sum())


@pytest.mark.parametrize("variant", sorted(oracle.VARIANTS))
def test_o2_intersection_counts_match_closed_forms(variant):
    bits = oracle.VARIANTS[variant]
    for g in _graphs():
        for dual in (0, 1):
            B = _side(g, dual)
            for s in (1, 2, 4):
                _, st_ = oracle.alg_h(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                      variant=bits, threads=2, keep=False)
                want = _intersections_closed_form(B, s, bits & oracle.H_PRUNE,
                                                  bits & oracle.H_VISITED)
                assert st_.intersections == want, (variant, s, dual)


@settings(max_examples=40, deadline=None)
@given(m=st.integers(1, 14), n=st.integers(1, 14), p=st.floats(0.05, 0.9),
       seed=st.integers(0, 2**31 - 1), s=st.integers(1, 5), variant=st.sampled_from(
           sorted(oracle.VARIANTS)))
def test_o2_on_drawn_graphs(m, n, p, seed, s, variant):
    rng = np.random.default_rng(seed)
    g = csr_from_dense((rng.random((m, n)) < p).astype(np.int64))
    for dual in (0, 1):
        B = _side(g, dual)
        a, b, w = pairs_from_dense(np.rint(B @ B.T).astype(np.int64), s)
        got, _ = oracle.alg_h(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                              variant=oracle.VARIANTS[variant])
        assert _same(got, a, b, w)


# ------------------------------------------------------------- filter_s

def test_filter_of_l1_is_ls():
    for g in _graphs():
        for dual in (0, 1):
            L1, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1, dual=dual)
            for s in (2, 3, 4, 6):
                direct, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual)
                f = oracle.filter_s(L1, s)
                assert _same(f, direct.a, direct.b, direct.w), (s, dual)
                # and from any L_s' in between
                mid, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, max(1, s - 1),
                                      dual=dual)
                f2 = oracle.filter_s(mid, s)
                assert _same(f2, direct.a, direct.b, direct.w)


# --------------------------------------------------- squeeze, adjacency

def _scipy_adjacency(L, n_items):
    M = sp.coo_matrix((np.asarray(L.w, dtype=np.int64), (L.a, L.b)), shape=(n_items, n_items))
    S = (M + M.T).tocsr()
    present = np.flatnonzero(np.diff(S.indptr) > 0)
    T = S[present][:, present].tocsr()
    T.sort_indices()
    return present, T


def test_squeeze_and_adjacency_match_scipy():
    for g in _graphs():
        for dual in (0, 1):
            N = g.n_vertices if dual else g.n_edges
            for s in (1, 2, 3):
                L, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual)
                old_id, Lq = oracle.squeeze(L, N)
                present, T = _scipy_adjacency(L, N)
                assert np.array_equal(old_id, present)
                # round trip: the new ids name the same items, order kept
                assert np.array_equal(old_id[Lq.a], L.a) and np.array_equal(old_id[Lq.b], L.b)
                assert np.all(np.diff(old_id) > 0)
                rp, col, w = oracle.adjacency(Lq, len(old_id))
                assert np.array_equal(rp, T.indptr) and np.array_equal(col, T.indices)
                assert np.array_equal(w, T.data)
                assert rp[-1] == 2 * len(L.a)


def test_squeeze_of_squeezed_is_identity():
    g = gen.uniform_hypergraph(200, 150, 2, 8, seed=9)
    L, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, 2)
    old_id, Lq = oracle.squeeze(L, g.n_edges)
    again, Lqq = oracle.squeeze(Lq, len(old_id))
    assert np.array_equal(again, np.arange(len(old_id)))
    assert _same(Lqq, Lq.a, Lq.b, Lq.w)


# ------------------------------------------------------------ components

def _canonical_labels(labels):
    """Relabel a partition by the smallest member of each part."""
    labels = np.asarray(labels)
    out = np.empty_like(labels)
    first = {}
    for x, l in enumerate(labels.tolist()):
        first.setdefault(l, x)
        out[x] = first[l]
    return out


def test_components_match_scipy():
    for g in _graphs():
        for dual in (0, 1):
            N = g.n_vertices if dual else g.n_edges
            for s in (1, 2, 3):
                L, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual)
                comp = oracle.components(N, L)
                M = sp.coo_matrix((np.ones(len(L.a)), (L.a, L.b)), shape=(N, N))
                _, lab = connected_components(M, directed=False)
                assert np.array_equal(comp, _canonical_labels(lab)), (s, dual)
                assert np.all(comp <= np.arange(N)) and np.array_equal(comp[comp], comp)


def test_components_closed_forms():
    # sunflower: every pair shares the core, so at s <= core one component
    g = gen.sunflower(9, 3, 4, seed=1)
    for s in (1, 2, 3):
        L, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s)
        assert np.array_equal(oracle.components(g.n_edges, L), np.zeros(g.n_edges))
    L, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, 4)
    assert np.array_equal(oracle.components(g.n_edges, L), np.arange(g.n_edges))
    # disjoint family: no pair, every item alone
    d = gen.from_sets([[0, 1], [2, 3, 4], [5], [6, 7]], 8)
    L, _ = oracle.wedge(d.row_ptr, d.col, d.n_edges, d.n_vertices, 1)
    assert np.array_equal(oracle.components(d.n_edges, L), np.arange(d.n_edges))
    # a path of overlapping sets: one component at s = 1, split at s = 2
    p = gen.from_sets([[0, 1], [1, 2], [2, 3, 4], [3, 4, 5], [9]], 10)
    L, _ = oracle.wedge(p.row_ptr, p.col, p.n_edges, p.n_vertices, 1)
    assert oracle.components(p.n_edges, L).tolist() == [0, 0, 0, 0, 4]
    L, _ = oracle.wedge(p.row_ptr, p.col, p.n_edges, p.n_vertices, 2)
    assert oracle.components(p.n_edges, L).tolist() == [0, 1, 2, 2, 4]


# --------------------------------------------------------------- relabel

@pytest.mark.parametrize("descending", [True, False])
def test_relabel_orders_sizes_and_maps_back(descending):
    for g in _graphs():
        for dual in (0, 1):
            N = g.n_vertices if dual else g.n_edges
            perm, rp2, col2, m2, n2 = oracle.relabel(g.row_ptr, g.col, g.n_edges, g.n_vertices,
                                                     dual, descending)
            assert np.array_equal(np.sort(perm), np.arange(N))
            size = (np.bincount(g.col, minlength=g.n_vertices) if dual
                    else np.diff(g.row_ptr))[perm]
            d = np.diff(size.astype(np.int64))
            assert np.all(d <= 0) if descending else np.all(d >= 0)
            ties = np.flatnonzero(d == 0)
            assert np.all(perm[ties] < perm[ties + 1])  # equal sizes keep id order
            # the relabeled hypergraph is the same hypergraph with items renamed
            B = _side(g, dual)
            B2 = _side(gen.Hypergraph(rp2, col2, m2, n2, {}), dual)
            assert np.array_equal(B2, B[perm])
            for s in (1, 2, 3):
                ref, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual)
                got, _ = oracle.naive(rp2, col2, m2, n2, s, dual=dual)
                back = oracle.map_back(got, perm)
                assert _same(back, ref.a, ref.b, ref.w), (s, dual, descending)
