"""Generators: deterministic per seed, valid CSR, realized statistics in range."""

from __future__ import annotations

import numpy as np

from paper_2010_11448_amd import gen


def valid_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int32 and col.dtype == np.int32
    assert rp[0] == 0 and (np.diff(rp) >= 0).all() and rp[-1] == len(col)
    if len(col):
        assert col.min() >= 0 and col.max() < g.n_vertices
    rows = np.repeat(np.arange(g.n_edges), np.diff(rp))
    same_row = rows[1:] == rows[:-1]
    assert (np.diff(col.astype(np.int64))[same_row] > 0).all()


def test_uniform_is_deterministic_and_valid():
    a = gen.uniform_2000(11)
    b = gen.uniform_2000(11)
    c = gen.uniform_2000(12)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert not np.array_equal(a.col, c.col)
    valid_csr(a)
    size = np.diff(a.row_ptr)
    assert size.min() >= 2 and size.max() <= 20 and 10 < size.mean() < 12
    assert a.n_edges == 2000 and a.n_vertices == 5000


def test_powerlaw_scaled_shape():
    g = gen.powerlaw_1m(scale=0.01)
    valid_csr(g)
    size = np.diff(g.row_ptr)
    assert size.min() >= 2 and size.max() <= 100
    deg = np.bincount(g.col, minlength=g.n_vertices)
    assert deg.max() > 20 * max(1.0, deg.mean())  # a skewed popularity law


def test_powerlaw_full_size_statistics():
    g = gen.powerlaw_1m()
    valid_csr(g)
    size = np.diff(g.row_ptr)
    deg = np.bincount(g.col, minlength=g.n_vertices)
    assert 7.4e6 < g.nnz < 8.0e6
    assert size.min() == 2 and size.max() <= 10_000
    assert 1.0e4 < deg.max() < 2.0e4
    assert 0.6 < (deg == 0).mean() < 0.72


def test_batch_law():
    sizes = gen.batch_sizes(n_graphs=512)
    assert len(sizes) == 512 and min(sizes) >= 1000 and max(sizes) <= 200_000
    assert 2.5e4 < np.mean(sizes) < 5.0e4
    item = gen.batch_graph(3, m_cap=3000)
    valid_csr(item.graph)
    assert 1 <= item.s <= 12 and item.graph.n_vertices == 2 * item.graph.n_edges


def test_serving_arrivals():
    q = gen.serving_arrivals(1024, 8, rate=200.0, duration_s=5.0)
    assert 800 < len(q) < 1200
    t = np.array([x.arrival_s for x in q])
    assert (np.diff(t) > 0).all() and t[-1] < 5.0
    assert all(1 <= x.s <= 16 and x.dual in (0, 1) and 0 <= x.graph_id < 1032 for x in q)
    big = np.mean([x.graph_id >= 1024 for x in q])
    assert 0.02 < big < 0.09


def test_planted_generators_are_valid():
    for g in (gen.sunflower(10, 3, 4, 1), gen.nested_chain(8, 3, 2),
              gen.planted_copies(gen.uniform_hypergraph(20, 30, 2, 5, 3), 2, 4),
              gen.random_small(40, 20, 8, 5)):
        valid_csr(g)
