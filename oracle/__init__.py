"""CPU oracle for s-line graphs -- test infrastructure, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``sline_oracle.c`` (plain C,
built with gcc) through ctypes and shares nothing with the HIP path.

Functions (items are hyperedges, or vertices when ``dual`` is set -- the dual
hypergraph of Sec. III, obtained here by the oracle's own counting-sort
transpose):

* ``naive(...)``  -- O1, the definition of L_s(H) (Sec. III) evaluated pair by
  pair as in the naive algorithm of Sec. IV-A; optionally for selected rows.
* ``wedge(...)``  -- O3, the alternative algorithm of Sec. IV-B with the
  visited array turned into an exact counter and degree-based pruning
  (Sec. IV-C); exact, validated against O1.
* ``alg_h(...)``  -- O2, the efficient algorithm with heuristics (Sec. IV-C)
  as printed, each heuristic a switch: the variants f0..f4 of Table III.
* ``transpose(...)`` -- the dual's item lists.

The pipeline stages after L_s (Table I), on an oracle edge list:

* ``filter_s(L, s)`` -- L_s from a weighted L_s' with s' <= s (Sec. III:
  L_s keeps the pairs of L_1 with w >= s, with the same w).
* ``squeeze(L, n_items)`` -- ID squeezing (Sec. IV-E): contiguous new ids for
  the items that occur in L, in the order of their original ids.
* ``adjacency(...)`` -- the line graph's adjacency as a symmetric CSR over
  the squeezed ids (Sec. IV-E: materializing it after squeezing).
* ``components(n_items, L)`` -- the s-connected components (Table I).
* ``relabel(...)`` -- relabel-by-degree (Sec. IV-F) and ``map_back``.

Each returns ``Pairs(a, b, w)`` (int32 numpy arrays, sorted by (a, b), a < b,
w >= s) and/or ``Stats`` (pair count, weight sum, order-independent digest,
wedges walked, intersections made).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sline_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Pairs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("a", ctypes.POINTER(ctypes.c_int32)),
                ("b", ctypes.POINTER(ctypes.c_int32)), ("w", ctypes.POINTER(ctypes.c_int32))]


class _Stats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("sum_w", ctypes.c_int64),
                ("digest", ctypes.c_uint64), ("wedges", ctypes.c_int64),
                ("intersections", ctypes.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i32p = P(ctypes.c_int32)
        lib.oracle_transpose.argtypes = [i32p, i32p, ctypes.c_int32, ctypes.c_int32, i32p, i32p]
        lib.oracle_naive_rows.argtypes = [i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, i32p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_int, P(_Pairs), P(_Stats)]
        lib.oracle_wedge_rows.argtypes = [i32p, i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                          i32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                          P(_Pairs), P(_Stats)]
        lib.oracle_alg_h_rows.argtypes = [i32p, i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, i32p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_int, P(_Pairs), P(_Stats)]
        lib.oracle_components.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int64, i32p]
        lib.oracle_free_pairs.argtypes = [P(_Pairs)]
        lib.oracle_mix.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_mix.restype = ctypes.c_uint64
        _lib = lib
    return _lib


@dataclass
class Pairs:
    a: np.ndarray
    b: np.ndarray
    w: np.ndarray

    def __len__(self) -> int:
        return len(self.a)

    def as_set(self) -> set:
        return set(zip(self.a.tolist(), self.b.tolist(), self.w.tolist()))


@dataclass
class Stats:
    n_pairs: int
    sum_w: int
    digest: int
    wedges: int
    intersections: int


def _ptr(x: np.ndarray | None):
    if x is None:
        return None
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def transpose(row_ptr, col, n_edges: int, n_vertices: int) -> tuple[np.ndarray, np.ndarray]:
    """Item lists of the dual: for each vertex, the ascending hyperedges containing it."""
    rp, cl = _i32(row_ptr), _i32(col)
    rpT = np.zeros(n_vertices + 1, dtype=np.int32)
    colT = np.zeros(max(1, int(rp[n_edges])), dtype=np.int32)
    rc = _load().oracle_transpose(_ptr(rp), _ptr(cl), n_edges, n_vertices, _ptr(rpT), _ptr(colT))
    if rc != 0:
        raise ValueError(f"oracle_transpose failed ({rc})")
    return rpT, colT[: int(rp[n_edges])]


def _items(row_ptr, col, n_edges, n_vertices, dual):
    rp, cl = _i32(row_ptr), _i32(col)
    if len(cl) == 0:
        cl = np.zeros(1, dtype=np.int32)
    if dual:
        rpT, colT = transpose(rp, cl, n_edges, n_vertices)
        if len(colT) == 0:
            colT = np.zeros(1, dtype=np.int32)
        return rpT, colT, n_vertices, rp, cl
    rpT, colT = transpose(rp, cl, n_edges, n_vertices)
    if len(colT) == 0:
        colT = np.zeros(1, dtype=np.int32)
    return rp, cl, n_edges, rpT, colT


def _finish(rc, pairs: _Pairs, st: _Stats, keep: bool):
    lib = _load()
    if rc != 0:
        raise RuntimeError(f"oracle failed ({rc})")
    stats = Stats(st.n_pairs, st.sum_w, st.digest, st.wedges, st.intersections)
    if not keep:
        return None, stats
    n = pairs.n
    if n:
        a = np.ctypeslib.as_array(pairs.a, shape=(n,)).copy()
        b = np.ctypeslib.as_array(pairs.b, shape=(n,)).copy()
        w = np.ctypeslib.as_array(pairs.w, shape=(n,)).copy()
    else:
        a = b = w = np.zeros(0, dtype=np.int32)
    lib.oracle_free_pairs(ctypes.byref(pairs))
    return Pairs(a, b, w), stats


def _rows_arg(rows):
    if rows is None:
        return None, 0
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    return r, len(r)


def naive(row_ptr, col, n_edges: int, n_vertices: int, s: int, dual: int = 0,
          rows=None, skip_small: bool = False, threads: int = 1, keep: bool = True):
    """O1: every pair (a, b > a) of items compared by a sorted merge.

    Returns ``(Pairs | None, Stats)``.  ``rows`` (ascending item ids) restricts
    the outer loop to those items; all b > a are still compared."""
    rp, cl, N, _, _ = _items(row_ptr, col, n_edges, n_vertices, dual)
    r, nr = _rows_arg(rows)
    pairs, st = _Pairs(), _Stats()
    rc = _load().oracle_naive_rows(_ptr(rp), _ptr(cl), N, s, int(skip_small), _ptr(r), nr,
                                   threads, int(keep), ctypes.byref(pairs), ctypes.byref(st))
    return _finish(rc, pairs, st, keep)


@dataclass
class Prepared:
    """Item lists and member lists of one side of a hypergraph, built once
    (the oracle's own counting-sort transpose) for many ``wedge`` calls."""

    rp: np.ndarray
    col: np.ndarray
    N: int
    rpT: np.ndarray
    colT: np.ndarray


def prepare(row_ptr, col, n_edges: int, n_vertices: int, dual: int = 0) -> Prepared:
    """The lists ``wedge`` walks for this side, for reuse across calls."""
    return Prepared(*_items(row_ptr, col, n_edges, n_vertices, dual))


def wedge(row_ptr, col, n_edges: int, n_vertices: int, s: int, dual: int = 0,
          rows=None, threads: int = 1, keep: bool = True, prepared: Prepared | None = None):
    """O3: wedge counting over shared members with exact counters.

    ``prepared`` (from ``prepare`` on the same graph and side) skips building
    the lists again; the graph arguments are then ignored."""
    if prepared is not None:
        rp, cl, N, rpT, colT = (prepared.rp, prepared.col, prepared.N, prepared.rpT,
                                prepared.colT)
    else:
        rp, cl, N, rpT, colT = _items(row_ptr, col, n_edges, n_vertices, dual)
    r, nr = _rows_arg(rows)
    pairs, st = _Pairs(), _Stats()
    rc = _load().oracle_wedge_rows(_ptr(rp), _ptr(cl), _ptr(rpT), _ptr(colT), N, s, _ptr(r), nr,
                                   threads, int(keep), ctypes.byref(pairs), ctypes.byref(st))
    return _finish(rc, pairs, st, keep)


def mix(a: int, b: int, w: int) -> int:
    """The digest term the oracle sums for one output triple."""
    return int(_load().oracle_mix(a, b, w))


# Heuristics of O2 (Sec. IV-C) and the variants of Table III.
H_PRUNE, H_VISITED, H_SHORT = 1, 2, 4
VARIANTS = {"f0": H_PRUNE | H_VISITED | H_SHORT, "f1": H_PRUNE, "f2": H_VISITED, "f3": H_SHORT,
            "f4": 0}


def alg_h(row_ptr, col, n_edges: int, n_vertices: int, s: int, dual: int = 0,
          variant: int = VARIANTS["f0"], rows=None, threads: int = 1, keep: bool = True):
    """O2: the heuristic algorithm with the given heuristics on; ``Stats``
    counts its set intersections."""
    rp, cl, N, rpT, colT = _items(row_ptr, col, n_edges, n_vertices, dual)
    r, nr = _rows_arg(rows)
    pairs, st = _Pairs(), _Stats()
    rc = _load().oracle_alg_h_rows(_ptr(rp), _ptr(cl), _ptr(rpT), _ptr(colT), N, s, int(variant),
                                   _ptr(r), nr, threads, int(keep), ctypes.byref(pairs),
                                   ctypes.byref(st))
    return _finish(rc, pairs, st, keep)


def filter_s(L: Pairs, s: int) -> Pairs:
    """The pairs of a weighted L_s' (s' <= s) with w >= s: L_s (Sec. III)."""
    keep = np.asarray(L.w) >= s
    return Pairs(np.asarray(L.a)[keep], np.asarray(L.b)[keep], np.asarray(L.w)[keep])


def squeeze(L: Pairs, n_items: int):
    """ID squeezing (Sec. IV-E).  Returns ``(old_id, Pairs)``: old_id[k] is the
    original id of new id k -- the items occurring in L, ascending -- and the
    pairs are L with both ids replaced by the new ones (still sorted, a < b)."""
    a = np.asarray(L.a, dtype=np.int64)
    b = np.asarray(L.b, dtype=np.int64)
    present = np.zeros(n_items, dtype=bool)
    present[a] = True
    present[b] = True
    old_id = np.flatnonzero(present).astype(np.int32)
    new_of_old = np.full(n_items, -1, dtype=np.int64)
    new_of_old[old_id] = np.arange(len(old_id))
    return old_id, Pairs(new_of_old[a].astype(np.int32), new_of_old[b].astype(np.int32),
                         np.asarray(L.w, dtype=np.int32).copy())


def adjacency(L: Pairs, n_nodes: int):
    """The adjacency of the undirected graph L over nodes 0..n_nodes-1 as a
    CSR: ``(row_ptr (int64, n_nodes + 1), col, w)``, every edge {a, b} in row
    a and in row b, each row in ascending neighbour order."""
    a = np.asarray(L.a, dtype=np.int64)
    b = np.asarray(L.b, dtype=np.int64)
    w = np.asarray(L.w, dtype=np.int32)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    ws = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_nodes), out=row_ptr[1:])
    return row_ptr, cols[order].astype(np.int32), ws[order]


def components(n_items: int, L: Pairs) -> np.ndarray:
    """s-connected components (Table I) of the graph L on items 0..n-1:
    comp[x] = the smallest item of x's component (an item with no pair is a
    component of its own)."""
    a = _i32(L.a)
    b = _i32(L.b)
    comp = np.zeros(max(n_items, 1), dtype=np.int32)
    rc = _load().oracle_components(n_items, _ptr(a) if len(a) else None,
                                   _ptr(b) if len(b) else None, len(a), _ptr(comp))
    if rc != 0:
        raise ValueError(f"oracle_components failed ({rc})")
    return comp[:n_items]


def relabel(row_ptr, col, n_edges: int, n_vertices: int, dual: int = 0,
            descending: bool = True):
    """Relabel-by-degree (Sec. IV-F) of the items of one side: new id k goes to
    the item of the k-th largest size (``descending``) or smallest, ties by
    original id.  Returns ``(perm, row_ptr', col', n_edges', n_vertices')``:
    perm[k] = original id of new item k, and the CSR of the same hypergraph
    with the items renumbered (rows reordered for the primal side; member ids
    of the vertex side rewritten, rows re-sorted, for the dual)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    cl = np.asarray(col, dtype=np.int64)
    if dual:
        size = np.bincount(cl, minlength=n_vertices)
    else:
        size = np.diff(rp)
    key = -size if descending else size
    perm = np.lexsort((np.arange(len(size)), key)).astype(np.int32)  # size order, then id
    if dual:
        new_of_old = np.empty(len(size), dtype=np.int64)
        new_of_old[perm] = np.arange(len(size))
        row = np.repeat(np.arange(n_edges), np.diff(rp))
        newc = new_of_old[cl]
        order = np.lexsort((newc, row))
        return perm, rp.astype(np.int32), newc[order].astype(np.int32), n_edges, n_vertices
    lens = np.diff(rp)[perm]
    nrp = np.zeros(n_edges + 1, dtype=np.int64)
    np.cumsum(lens, out=nrp[1:])
    ncol = np.concatenate([cl[rp[i]:rp[i + 1]] for i in perm]) if n_edges else cl[:0]
    return perm, nrp.astype(np.int32), ncol.astype(np.int32), n_edges, n_vertices


def map_back(L: Pairs, perm) -> Pairs:
    """Pairs of relabeled items in original ids: (perm[a], perm[b]) ordered so
    the smaller id comes first, then sorted by (a, b)."""
    perm = np.asarray(perm, dtype=np.int64)
    x = perm[np.asarray(L.a, dtype=np.int64)]
    y = perm[np.asarray(L.b, dtype=np.int64)]
    a, b = np.minimum(x, y), np.maximum(x, y)
    order = np.lexsort((b, a))
    return Pairs(a[order].astype(np.int32), b[order].astype(np.int32),
                 np.asarray(L.w, dtype=np.int32)[order])
