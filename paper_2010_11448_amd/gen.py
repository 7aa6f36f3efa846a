"""Seeded synthetic hypergraph generators.

This module draws inputs only; it holds none of the s-overlap arithmetic.  It is
the one module that both the CPU oracle side (tests, golden-value scripts) and
the device path (bench, GPU tests) use, so it must stay free of any step of the
method.

A hypergraph is returned as an int32 incidence CSR with rows = hyperedges:
``row_ptr[m+1]`` and ``col[nnz]``, every row strictly increasing.  The paper's
definition (Sec. III) allows an indexed family of subsets of V with empty,
singleton and duplicate hyperedges and isolated vertices; the generators below
produce all of these where the size law allows it.

Random numbers come from ``numpy.random.PCG64(seed).random_raw()`` turned into
53-bit uniforms; every distribution is sampled by our own inverse-CDF or
Box-Muller code so that numpy's distribution methods (which may change between
versions) are never used.

Workloads (sizes from the benchmark configurations):

* uniform   -- m hyperedges over n vertices, sizes uniform on [lo, hi],
               members uniform without replacement (2000 x 5000, sizes 2..20).
* powerlaw  -- m = 1e6 hyperedges over n = 2e6 vertices; hyperedge sizes
               truncated Zipf(2.2) on [2, 1e4]; vertex popularity t_v drawn iid
               from truncated Zipf(1.8) on [1, 1e5]; members drawn with
               probability proportional to t_v, without replacement.
* dual of powerlaw -- same arrays, roles swapped by the caller (dual flag).
* batch     -- 512 graphs, m_g = clip(lognormal(ln 2e4, 1.2), 1e3, 2e5),
               n_g = 2 m_g, sizes truncated Zipf(2.2) on [2, 2000], uniform
               members, per-graph s uniform on {1..12}.
* serving   -- a resident catalog drawn from the batch law plus a few
               powerlaw-sized graphs, queried by Poisson arrivals.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GEN_VERSION = 1

_MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One step of the SplitMix64 output function (Steele, Lea, Flood 2014)."""
    x = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return (z ^ (z >> 31)) & _MASK64


def sub_seed(base: int, index: int) -> int:
    """Independent per-item seed derived from (base, index)."""
    return splitmix64(splitmix64(base & _MASK64) ^ (index & _MASK64))


class Stream:
    """A seeded source of raw 64-bit words and the draws built on them."""

    def __init__(self, seed: int):
        self._bg = np.random.PCG64(seed)

    def raw(self, size: int) -> np.ndarray:
        return self._bg.random_raw(size).astype(np.uint64)

    def uniform(self, size: int) -> np.ndarray:
        """Uniforms on [0, 1) with 53 random bits each."""
        return (self.raw(size) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def integers(self, lo: int, hi: int, size: int) -> np.ndarray:
        """Integers uniform on the closed range [lo, hi]."""
        span = hi - lo + 1
        k = np.floor(self.uniform(size) * span).astype(np.int64)
        return lo + np.minimum(k, span - 1)

    def normal(self, size: int) -> np.ndarray:
        """Standard normals by the Box-Muller transform."""
        u1 = self.uniform(size)
        u2 = self.uniform(size)
        u1 = np.where(u1 <= 0.0, 2.0 ** -53, u1)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)

    def exponential(self, rate: float, size: int) -> np.ndarray:
        u = self.uniform(size)
        return -np.log1p(-u) / rate


def zipf_cdf(alpha: float, lo: int, hi: int) -> np.ndarray:
    """CDF table of the truncated Zipf law P(k) proportional to k^-alpha on [lo, hi]."""
    k = np.arange(lo, hi + 1, dtype=np.float64)
    pmf = k ** (-alpha)
    cdf = np.cumsum(pmf)
    return cdf / cdf[-1]


def sample_cdf(stream: Stream, cdf: np.ndarray, lo: int, size: int) -> np.ndarray:
    """Inverse-CDF sampling over a table whose first entry is value ``lo``."""
    u = stream.uniform(size)
    idx = np.searchsorted(cdf, u, side="right")
    return lo + np.minimum(idx, len(cdf) - 1)


def _draw_rows(stream: Stream, sizes: np.ndarray, n: int,
               weight_cdf: np.ndarray | None) -> tuple[np.ndarray, np.ndarray]:
    """Draw each row's members without replacement and return a sorted CSR.

    Members are drawn from ``weight_cdf`` (cumulative vertex weights) or
    uniformly when it is None; a member repeated inside a row is redrawn until
    the row holds distinct members, then every row is sorted.
    """
    m = len(sizes)
    sizes = sizes.astype(np.int64)
    if np.any(sizes > n):
        raise ValueError("a hyperedge is larger than the vertex set")
    nnz = int(sizes.sum())
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=row_ptr[1:])
    row = np.repeat(np.arange(m, dtype=np.int64), sizes)

    def draw(k):
        if weight_cdf is None:
            return stream.integers(0, n - 1, k)
        u = stream.uniform(k)
        return np.minimum(np.searchsorted(weight_cdf, u, side="right"), n - 1)

    v = draw(nnz).astype(np.int64)
    while True:
        key = row * n + v
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.flatnonzero(ks[1:] == ks[:-1]) + 1
        if dup.size == 0:
            break
        pos = np.sort(order[dup])
        v[pos] = draw(pos.size)
    col = np.empty(nnz, dtype=np.int64)
    col[:] = v[np.argsort(row * n + v, kind="stable")]
    return row_ptr.astype(np.int32), col.astype(np.int32)


@dataclass
class Hypergraph:
    """Incidence CSR (rows = hyperedges) plus the recipe that drew it."""

    row_ptr: np.ndarray
    col: np.ndarray
    n_edges: int
    n_vertices: int
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def uniform_hypergraph(m: int, n: int, size_lo: int, size_hi: int, seed: int) -> Hypergraph:
    """Sizes uniform on [size_lo, size_hi]; members uniform without replacement."""
    st = Stream(seed)
    sizes = st.integers(size_lo, size_hi, m)
    rp, col = _draw_rows(st, sizes, n, None)
    return Hypergraph(rp, col, m, n, dict(kind="uniform", m=m, n=n, size_lo=size_lo,
                                          size_hi=size_hi, seed=seed, gen_version=GEN_VERSION))


def powerlaw_hypergraph(m: int, n: int, size_alpha: float, size_lo: int, size_hi: int,
                        pop_alpha: float, pop_hi: int, seed: int) -> Hypergraph:
    """Zipf hyperedge sizes; members drawn proportional to Zipf vertex popularity."""
    st = Stream(seed)
    sizes = sample_cdf(st, zipf_cdf(size_alpha, size_lo, size_hi), size_lo, m)
    sizes = np.minimum(sizes, n)
    if pop_hi > 0:
        t = sample_cdf(st, zipf_cdf(pop_alpha, 1, pop_hi), 1, n).astype(np.float64)
        wcdf = np.cumsum(t)
        wcdf /= wcdf[-1]
    else:
        wcdf = None
    rp, col = _draw_rows(st, sizes, n, wcdf)
    return Hypergraph(rp, col, m, n, dict(kind="powerlaw", m=m, n=n, size_alpha=size_alpha,
                                          size_lo=size_lo, size_hi=size_hi, pop_alpha=pop_alpha,
                                          pop_hi=pop_hi, seed=seed, gen_version=GEN_VERSION))


def zipf_uniform_hypergraph(m: int, n: int, size_alpha: float, size_lo: int, size_hi: int,
                            seed: int) -> Hypergraph:
    """Zipf hyperedge sizes with uniform members (the batch-workload law)."""
    g = powerlaw_hypergraph(m, n, size_alpha, size_lo, size_hi, 0.0, 0, seed)
    g.meta["kind"] = "zipf_uniform"
    return g


# ---------------------------------------------------------------- workloads

UNIFORM_SEEDS = (11, 12, 13)
POWERLAW_SEED = 21
BATCH_SEED = 41
SERVE_SEED = 51

UNIFORM_S = tuple(range(1, 9))
POWERLAW_S = (1, 2, 4, 8, 16)
DUAL_S = (2, 8, 32)


def uniform_2000(seed: int = 11) -> Hypergraph:
    """2,000 hyperedges over 5,000 vertices, sizes uniform on [2, 20]."""
    g = uniform_hypergraph(2000, 5000, 2, 20, seed)
    g.meta["workload"] = "uniform_2000x5000"
    return g


def powerlaw_1m(seed: int = POWERLAW_SEED, scale: float = 1.0) -> Hypergraph:
    """1e6 hyperedges over 2e6 vertices with power-law sizes and popularity.

    ``scale`` shrinks m and n (and the clips) together for smaller stand-ins of
    the same shape.
    """
    m = max(1, int(round(1_000_000 * scale)))
    n = max(1, int(round(2_000_000 * scale)))
    size_hi = max(2, min(10_000, int(round(10_000 * scale)) if scale < 1 else 10_000))
    pop_hi = max(1, min(100_000, int(round(100_000 * scale)) if scale < 1 else 100_000))
    g = powerlaw_hypergraph(m, n, 2.2, 2, size_hi, 1.8, pop_hi, seed)
    g.meta["workload"] = "powerlaw_1Mx2M" if scale == 1.0 else f"powerlaw_scaled_{scale:g}"
    return g


@dataclass
class BatchItem:
    graph: Hypergraph
    s: int
    dual: int = 0


def batch_sizes(seed: int = BATCH_SEED, n_graphs: int = 512) -> list[int]:
    """Hyperedge counts m_g = clip(lognormal(ln 2e4, 1.2), 1e3, 2e5)."""
    out = []
    for g in range(n_graphs):
        st = Stream(sub_seed(seed, g))
        z = float(st.normal(1)[0])
        mg = int(round(math.exp(math.log(20_000) + 1.2 * z)))
        out.append(min(200_000, max(1_000, mg)))
    return out


def batch_graph(g: int, seed: int = BATCH_SEED, m_cap: int | None = None) -> BatchItem:
    """Graph ``g`` of the batch workload with its own s on {1..12}."""
    st = Stream(sub_seed(seed, g))
    z = float(st.normal(1)[0])
    mg = int(round(math.exp(math.log(20_000) + 1.2 * z)))
    mg = min(200_000, max(1_000, mg))
    if m_cap is not None:
        mg = min(mg, m_cap)
    s = int(st.integers(1, 12, 1)[0])
    gs = sub_seed(seed ^ 0x5EED, g)
    hg = zipf_uniform_hypergraph(mg, 2 * mg, 2.2, 2, 2000, gs)
    hg.meta["workload"] = "batch_lognormal"
    hg.meta["index"] = g
    hg.meta["s"] = s
    return BatchItem(hg, s, 0)


def batch_workload(n_graphs: int = 512, seed: int = BATCH_SEED,
                   m_cap: int | None = None) -> list[BatchItem]:
    return [batch_graph(g, seed, m_cap) for g in range(n_graphs)]


@dataclass
class Query:
    arrival_s: float
    graph_id: int
    s: int
    dual: int


def serving_arrivals(n_catalog_small: int, n_catalog_large: int, rate: float = 200.0,
                     duration_s: float = 60.0, seed: int = SERVE_SEED,
                     large_frac: float = 0.05) -> list[Query]:
    """Poisson arrivals; each query picks a catalog graph, s on {1..16} and a side.

    Catalog ids ``0..n_catalog_small-1`` are batch-law graphs and the following
    ``n_catalog_large`` ids are powerlaw-sized graphs.
    """
    st = Stream(sub_seed(seed, 0xA77))
    out: list[Query] = []
    t = 0.0
    while True:
        t += float(st.exponential(rate, 1)[0])
        if t >= duration_s:
            break
        u = float(st.uniform(1)[0])
        if n_catalog_large > 0 and u < large_frac:
            gid = n_catalog_small + int(st.integers(0, n_catalog_large - 1, 1)[0])
        else:
            gid = int(st.integers(0, n_catalog_small - 1, 1)[0])
        s = int(st.integers(1, 16, 1)[0])
        dual = int(st.integers(0, 1, 1)[0])
        out.append(Query(t, gid, s, dual))
    return out


# ------------------------------------------------------- planted structures

def from_sets(sets: list[list[int]], n: int) -> Hypergraph:
    """CSR from an explicit list of member lists (each is sorted and deduplicated)."""
    rows = [sorted(set(int(x) for x in e)) for e in sets]
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in r], dtype=np.int32)
    return Hypergraph(rp, col, len(rows), n, dict(kind="explicit"))


def sunflower(n_petals: int, core: int, petal: int, seed: int) -> Hypergraph:
    """Hyperedges sharing one core of ``core`` vertices, petals disjoint, ids shuffled."""
    st = Stream(seed)
    n = core + n_petals * petal
    perm = np.argsort(st.uniform(n), kind="stable")
    core_ids = perm[:core]
    sets = []
    for p in range(n_petals):
        pet = perm[core + p * petal: core + (p + 1) * petal]
        sets.append(list(core_ids) + list(pet))
    return from_sets(sets, n)


def planted_copies(base: Hypergraph, copies: int, seed: int) -> Hypergraph:
    """Each hyperedge of ``base`` repeated ``copies`` times, the order shuffled."""
    st = Stream(seed)
    rows = [base.col[base.row_ptr[i]:base.row_ptr[i + 1]].tolist() for i in range(base.n_edges)]
    rows = rows * copies
    order = np.argsort(st.uniform(len(rows)), kind="stable")
    return from_sets([rows[i] for i in order], base.n_vertices)


def nested_chain(n_sets: int, step: int, seed: int) -> Hypergraph:
    """Sets e_0 within e_1 within ... (prefixes of one shuffled vertex order), ids shuffled."""
    st = Stream(seed)
    n = n_sets * step
    perm = np.argsort(st.uniform(n), kind="stable")
    sets = [list(perm[:(k + 1) * step]) for k in range(n_sets)]
    order = np.argsort(st.uniform(n_sets), kind="stable")
    return from_sets([sets[i] for i in order], n)


def random_small(m: int, n: int, max_size: int, seed: int, p_empty: float = 0.1) -> Hypergraph:
    """Tiny hypergraphs with empty, singleton and duplicate rows for brute-force checks."""
    st = Stream(seed)
    sets = []
    for i in range(m):
        if sets and st.uniform(1)[0] < 0.1:
            sets.append(list(sets[int(st.integers(0, len(sets) - 1, 1)[0])]))
            continue
        if st.uniform(1)[0] < p_empty:
            sets.append([])
            continue
        k = int(st.integers(1, max(1, min(max_size, n)), 1)[0])
        pick = np.argsort(st.uniform(n), kind="stable")[:k]
        sets.append(pick.tolist())
    return from_sets(sets, n)


# ------------------------------------------------- parallel generation

def make(kind: str, *args, **kw) -> Hypergraph:
    """A workload graph by name: ``powerlaw_1m``, ``batch_graph`` (its
    Hypergraph only), ``uniform_2000``."""
    if kind == "powerlaw_1m":
        return powerlaw_1m(*args, **kw)
    if kind == "batch_graph":
        return batch_graph(*args, **kw).graph
    if kind == "uniform_2000":
        return uniform_2000(*args, **kw)
    raise ValueError(kind)


def _make_spec(spec):
    kind, args, kw = spec
    return make(kind, *args, **kw)


def make_many(specs: list, workers: int = 1) -> list[Hypergraph]:
    """``make`` over (kind, args, kwargs) specs, in fresh worker processes when
    ``workers`` > 1 (every draw is seeded per graph, so the result does not
    depend on the number of workers).  Call it before the process touches a
    GPU: the workers are started with ``spawn``."""
    if workers <= 1 or len(specs) <= 1:
        return [_make_spec(s) for s in specs]
    import concurrent.futures as cf
    import multiprocessing as mp

    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_make_spec, specs, chunksize=max(1, len(specs) // (4 * workers))))
