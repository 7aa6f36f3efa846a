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
* ``transpose(...)`` -- the dual's item lists.

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
