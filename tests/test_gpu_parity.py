"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bar: bit-exact -- the output is integer (ids and overlaps), so every element
of a, b and w must equal the oracle's, in the same canonical (a, b) order.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2010_11448_amd import gen

from helpers import assert_same, check_canonical_torch, digest_torch, to_device

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


def _check(ctx, dev, g, s, dual, what):
    print(f"case: {what} m={g.n_edges} n={g.n_vertices} s={s} dual={dual}", flush=True)
    rp, col = to_device(g, dev)
    L = ctx.build(rp, col, g.n_vertices, s, dual)
    ref, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
    assert_same(L, ref, f"{what} s={s} dual={dual}")
    return L


@pytest.mark.parametrize("seed", gen.UNIFORM_SEEDS)
@pytest.mark.parametrize("dual", [0, 1])
def test_uniform_2000_all_s(ctx, dev, seed, dual):
    g = gen.uniform_2000(seed)
    for s in gen.UNIFORM_S:
        _check(ctx, dev, g, s, dual, f"uniform_2000 seed={seed}")


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_random_small_with_duplicates_and_empty_rows(ctx, dev, seed):
    g = gen.random_small(60, 40, 12, seed)
    for dual in (0, 1):
        for s in (1, 2, 3, 5, 13):
            _check(ctx, dev, g, s, dual, f"random_small seed={seed}")


def test_planted_structures(ctx, dev):
    sun = gen.sunflower(300, 6, 5, seed=3)
    for s in (1, 5, 6, 7):
        _check(ctx, dev, sun, s, 0, "sunflower")
    nest = gen.nested_chain(40, 7, seed=4)
    for s in (1, 7, 100, 200, 280, 281):
        _check(ctx, dev, nest, s, 0, "nested")
        _check(ctx, dev, nest, s, 1, "nested")
    cp = gen.planted_copies(gen.uniform_hypergraph(200, 300, 4, 12, seed=9), 3, seed=10)
    for s in (1, 4, 8, 12):
        _check(ctx, dev, cp, s, 0, "copies")


def test_powerlaw_scaled(ctx, dev):
    """A 1/50-scale power-law graph: heavy items, hub members, many passes."""
    g = gen.powerlaw_1m(scale=0.02)
    for dual, ss in ((0, (1, 2, 4, 8, 16)), (1, (2, 8, 32))):
        for s in ss:
            print(f"case: powerlaw 0.02 s={s} dual={dual}", flush=True)
            rp, col = to_device(g, dev)
            L = ctx.build(rp, col, g.n_vertices, s, dual)
            ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
            assert_same(L, ref, f"powerlaw0.02 s={s} dual={dual}")


def test_edge_cases(ctx, dev):
    import torch
    from paper_2010_11448_amd import sline

    # no hyperedges
    rp = torch.zeros(1, dtype=torch.int32, device=dev)
    col = torch.zeros(0, dtype=torch.int32, device=dev)
    assert len(ctx.build(rp, col, 5, 1, 0)) == 0
    assert len(ctx.build(rp, col, 5, 1, 1)) == 0
    # all rows empty
    rp = torch.zeros(4, dtype=torch.int32, device=dev)
    assert len(ctx.build(rp, col, 3, 1, 0)) == 0
    # one item
    g = gen.from_sets([[0, 1, 2]], 3)
    _check(ctx, dev, g, 1, 0, "single")
    _check(ctx, dev, g, 1, 1, "single dual")
    # s above every size, up to the largest int32
    g = gen.uniform_2000(11)
    rpd, cold = to_device(g, dev)
    assert len(ctx.build(rpd, cold, g.n_vertices, 21, 0)) == 0
    for dual in (0, 1):
        assert len(ctx.build(rpd, cold, g.n_vertices, 2 ** 31 - 1, dual)) == 0
    # in a batch beside a graph with pairs
    both = ctx.build_batch([(rpd, cold, g.n_vertices)] * 2, [2 ** 31 - 1, 2], [0, 0])
    assert len(both[0]) == 0
    ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, 2, dual=0, threads=8)
    assert_same(both[1], ref, "batch beside s = 2^31 - 1")
    # identical rows
    g = gen.from_sets([[1, 3, 5]] * 5 + [[0], []], 6)
    for s in (1, 3, 4):
        _check(ctx, dev, g, s, 0, "identical")
        _check(ctx, dev, g, s, 1, "identical dual")


def test_invalid_inputs(ctx, dev):
    import torch
    from paper_2010_11448_amd import sline

    def bad(rp, col, n, s=1, dual=0):
        with pytest.raises(sline.SlineError) as ei:
            ctx.build(torch.tensor(rp, dtype=torch.int32, device=dev),
                      torch.tensor(col, dtype=torch.int32, device=dev), n, s, dual)
        assert ei.value.status == sline.SLINE_EINVAL

    bad([0, 2, 4], [0, 1, 1, 1], 3)           # repeated member in a row
    bad([0, 2, 4], [1, 0, 0, 2], 3)           # decreasing row
    bad([0, 2, 4], [0, 3, 0, 1], 3)           # member out of range
    bad([0, 2, 4], [0, -1, 0, 1], 3)          # negative member
    bad([1, 2, 4], [0, 1, 0, 1], 3)           # row_ptr[0] != 0
    bad([0, 3, 2], [0, 1, 2], 3)              # decreasing row_ptr
    bad([0, 1, 2], [0, 1], 2, s=0)            # s < 1
    bad([0, 1, 2], [0, 1], 2, dual=2)         # bad dual flag

    # sizes, pointers and output buffers, through the C-ABI itself
    rp = torch.tensor([0, 2], dtype=torch.int32, device=dev)
    col = torch.tensor([0, 1], dtype=torch.int32, device=dev)
    buf = torch.zeros(3, dtype=torch.int32, device=dev)
    R, C = rp.data_ptr(), col.data_ptr()
    lib_owned = sline.sline_edges(0, 0, None, None, None)
    cases = [
        ("negative n_edges", sline.sline_csr(R, C, -1, 2), lib_owned),
        ("negative n_vertices", sline.sline_csr(R, C, 1, -1), lib_owned),
        ("row_ptr NULL", sline.sline_csr(None, C, 1, 2), lib_owned),
        ("col_idx NULL with members", sline.sline_csr(R, None, 1, 2), lib_owned),
        ("members but no vertices", sline.sline_csr(R, C, 1, 0), lib_owned),
        ("negative capacity", sline.sline_csr(R, C, 1, 2), sline.sline_edges(0, -1, None, None, None)),
        ("capacity without buffers", sline.sline_csr(R, C, 1, 2),
         sline.sline_edges(0, 1, buf.data_ptr(), None, None)),
    ]
    for what, H, out in cases:
        print(f"case: invalid {what}", flush=True)
        assert sline.sline_build(ctx.ctx, H, 1, 0, 0, out) == sline.SLINE_EINVAL, what
    # the context still builds after every refusal
    g = gen.from_sets([[0, 1], [1, 2], [0, 1, 2]], 3)
    _check(ctx, dev, g, 1, 0, "after invalid inputs")


def test_capacity_protocol(ctx, dev):
    """ECAPACITY reports the size and a retry writes the same result."""
    import torch
    from paper_2010_11448_amd import sline

    g = gen.uniform_2000(12)
    rp, col = to_device(g, dev)
    H = sline.Context.csr(rp, col, g.n_vertices)
    small = torch.zeros(3 * 10, dtype=torch.int32, device=dev)
    out = sline.sline_edges(0, 10, small[0:10].data_ptr(), small[10:20].data_ptr(),
                            small[20:30].data_ptr())
    st = sline.sline_build(ctx.ctx, H, 1, 0, 0, out)
    assert st == sline.SLINE_ECAPACITY
    need = int(out.n_pairs)
    ref, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    assert need == len(ref)
    buf = torch.zeros(3 * need, dtype=torch.int32, device=dev)
    out = sline.sline_edges(0, need, buf[0:need].data_ptr(), buf[need:2 * need].data_ptr(),
                            buf[2 * need:].data_ptr())
    assert sline.sline_build(ctx.ctx, H, 1, 0, 0, out) == sline.SLINE_OK
    L = sline.LineGraph(buf[0:need], buf[need:2 * need], buf[2 * need:])
    assert_same(L, ref, "capacity retry")
    # library-allocated output, freed by the library
    out = sline.sline_edges(0, 0, None, None, None)
    assert sline.sline_build(ctx.ctx, H, 2, 0, 0, out) == sline.SLINE_OK
    assert out.n_pairs == oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 2)[1].n_pairs
    assert sline.sline_edges_free(ctx.ctx, out) == sline.SLINE_OK
    assert out.a is None and out.n_pairs == 0


def test_deterministic_repeat(ctx, dev):
    g = gen.powerlaw_1m(scale=0.01)
    rp, col = to_device(g, dev)
    for s, dual in ((1, 0), (2, 1)):
        L1 = ctx.build(rp, col, g.n_vertices, s, dual)
        L2 = ctx.build(rp, col, g.n_vertices, s, dual)
        import torch
        assert torch.equal(L1.a, L2.a) and torch.equal(L1.b, L2.b) and torch.equal(L1.w, L2.w)
        check_canonical_torch(L1.a, L1.b, L1.w, s)


def test_stats_match_oracle(ctx, dev):
    g = gen.powerlaw_1m(scale=0.01)
    rp, col = to_device(g, dev)
    for s, dual in ((1, 0), (4, 0), (2, 1)):
        L = ctx.build(rp, col, g.n_vertices, s, dual)
        st = ctx.stats()
        _, ost = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                              threads=8, keep=False)
        assert st["wedges"] == ost.wedges
        assert st["n_pairs"] == ost.n_pairs == len(L)
        assert digest_torch(L.a, L.b, L.w) == ost.digest


def test_wide_items_and_long_member_lists(ctx, dev):
    """Items with tens of thousands of members: packed counters need more
    count bits (narrower key ranges, forced range splits) and members beyond
    the per-thread cursor window; checked against the wedge oracle."""
    st = gen.Stream(77)
    m, n = 300_000, 400_000
    sets = [sorted(set(st.integers(0, n - 1, 2).tolist())) for _ in range(m)]
    for pos in (5, 150_000, 299_990):
        sets[pos] = sorted(set(st.integers(0, n - 1, 30_000).tolist()))
    sets[7] = sets[5][:20_000]
    g = gen.from_sets(sets, n)
    rp, col = to_device(g, dev)
    for dual, s in ((0, 1), (0, 2), (0, 3), (1, 3), (1, 4)):
        print(f"case: wide items s={s} dual={dual}", flush=True)
        L = ctx.build(rp, col, g.n_vertices, s, dual)
        ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
        assert_same(L, ref, f"wide s={s} dual={dual}")


def test_tuning_changes_speed_not_result(ctx, dev):
    """Launch parameters (including a staging pool too small for the result,
    which forces tasks to be counted again) never change the output."""
    g = gen.powerlaw_1m(scale=0.01)
    rp, col = to_device(g, dev)
    base = ctx.tuning()
    refs = {}
    for s, dual in ((1, 0), (2, 0), (2, 1)):
        refs[(s, dual)], _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s,
                                          dual=dual, threads=8)
    variants = [dict(stage_max_bytes=0), dict(stage_max_bytes=1 << 20),
                dict(task_wedges=64, group_parts=1), dict(task_wedges=20000, group_parts=64),
                dict(small_max_wedges=0), dict(light_len=0), dict(light_len=64),
                dict(small_grid_per_cu=1, task_grid_per_cu=1),
                # every LDS table size the counting kernels are built for
                dict(small_slots=512, small_max_wedges=256), dict(small_slots=2048),
                dict(small_slots=2048, small_max_wedges=1024), dict(task_slots=4480),
                dict(task_slots=13440, task_grid_per_cu=2),
                dict(task_slots=17920, task_grid_per_cu=2, task_wedges=10000),
                dict(task_slots=4480, dense_min_wedges=0, task_wedges=64),
                # items counted one per lane: off, and with a small pool
                dict(tiny_max_wedges=0), dict(tiny_max_wedges=4, stage_max_bytes=1 << 20)]
    try:
        for v in variants:
            ctx.set_tuning(**{**base, **v})
            for (s, dual), ref in refs.items():
                print(f"case: tuning {v} s={s} dual={dual}", flush=True)
                L = ctx.build(rp, col, g.n_vertices, s, dual)
                assert_same(L, ref, f"tuning {v} s={s} dual={dual}")
    finally:
        ctx.set_tuning(**base)


def _claim_graph(seed: int = 5):
    """Hyperedges 0..9 each hold vertices 0..399, which lie in 240, 410 and 8
    other hyperedges (150, 150 and 100 of them); 6000 more vertices lie in one
    random hyperedge each (4000 hyperedges)."""
    rng = np.random.default_rng(seed)
    m, core = 4000, 400
    deg = np.concatenate([np.full(150, 240), np.full(150, 410), np.full(100, 8)])
    rows = [np.repeat(np.arange(10, dtype=np.int64), core)]
    cols = [np.tile(np.arange(core, dtype=np.int64), 10)]
    for v in range(core):
        rows.append(rng.choice(np.arange(10, m), size=int(deg[v]), replace=False))
        cols.append(np.full(int(deg[v]), v, np.int64))
    rows.append(rng.integers(10, m, size=6000))
    cols.append(np.arange(core, core + 6000, dtype=np.int64))
    key = np.unique(np.concatenate(rows) * 10 ** 6 + np.concatenate(cols))
    r, c = key // 10 ** 6, key % 10 ** 6
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return gen.Hypergraph(np.cumsum(rp).astype(np.int32), c.astype(np.int32), m, core + 6000,
                          dict(kind="claims"))


@pytest.mark.parametrize("tune", [dict(light_len=0, task_wedges=1 << 20), dict(light_len=0),
                                  dict()])
def test_piece_claims_past_capacity(ctx, dev, tune):
    """Ten items of 400 members whose runs ask for one to three pieces each
    (about 850 in all when the item is one task): more than a workgroup's
    run arrays hold, so reservations fail, one of them part-way through the
    arrays (its slots are left as empty pieces), and their members are walked
    by their lane.  The result equals the oracle's."""
    g = _claim_graph()
    rp, col = to_device(g, dev)
    base = ctx.tuning()
    ctx.set_tuning(**{**base, **tune})
    try:
        for s, dual in ((1, 0), (2, 0), (5, 0), (2, 1)):
            print(f"case: claims {tune} s={s} dual={dual}", flush=True)
            L = ctx.build(rp, col, g.n_vertices, s, dual)
            ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                  threads=8)
            assert_same(L, ref, f"claims {tune} s={s} dual={dual}")
    finally:
        ctx.set_tuning(**base)


@pytest.mark.parametrize("tiny", [10, 4, 0])
def test_tiny_items_one_per_lane(ctx, dev, tiny):
    """Builds with enough items (>= 32768) count their tiny items one per lane;
    the result equals the oracle with that path at two cost limits and off."""
    g = gen.uniform_hypergraph(50_000, 60_000, 2, 9, seed=31)
    rp, col = to_device(g, dev)
    base = ctx.tuning()
    ctx.set_tuning(**{**base, "tiny_max_wedges": tiny})
    try:
        for dual, s in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3)):
            print(f"case: tiny={tiny} s={s} dual={dual}", flush=True)
            L = ctx.build(rp, col, g.n_vertices, s, dual)
            ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                  threads=8)
            assert_same(L, ref, f"tiny={tiny} s={s} dual={dual}")
    finally:
        ctx.set_tuning(**base)


def test_tuning_rejects_out_of_range(ctx):
    from paper_2010_11448_amd import sline
    base = ctx.tuning()
    for bad in (dict(task_wedges=1), dict(small_max_wedges=100000), dict(group_parts=0),
                dict(stage_max_bytes=-1), dict(small_slots=768), dict(task_slots=9000),
                dict(small_slots=512, small_max_wedges=512), dict(tiny_max_wedges=11)):
        with pytest.raises(sline.SlineError):
            ctx.set_tuning(**{**base, **bad})
    assert ctx.tuning() == base


@pytest.mark.parametrize("n", [1, 16, 17, 256, 257, 70_000, 3_000_000])
def test_transpose_digit_boundaries(ctx, dev, n):
    """Member counts on both sides of the transpose's 4-bit digit boundaries
    (one to six radix passes), duplicate rows included (n = 1), both sides."""
    g = gen.uniform_hypergraph(300, n, 1, min(n, 12), 60 + n % 97)
    rp, col = to_device(g, dev)
    for dual in (0, 1):
        for s in (1, 2):
            print(f"case: transpose n={n} s={s} dual={dual}", flush=True)
            L = ctx.build(rp, col, g.n_vertices, s, dual)
            ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual,
                                  threads=8)
            assert_same(L, ref, f"n={n} s={s} dual={dual}")


def test_pairs_only_flag(ctx, dev):
    """SLINE_NO_WEIGHTS: the same pairs, w neither needed nor written."""
    import torch
    from paper_2010_11448_amd import sline

    for g, cases in ((gen.uniform_2000(11), ((1, 0), (2, 1), (3, 0))),
                     (gen.powerlaw_1m(scale=0.01), ((1, 0), (4, 0), (2, 1)))):
        rp, col = to_device(g, dev)
        for s, dual in cases:
            print(f"case: pairs only s={s} dual={dual}", flush=True)
            L = ctx.build(rp, col, g.n_vertices, s, dual, sline.SLINE_NO_WEIGHTS)
            assert L.w is None
            ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
            assert np.array_equal(L.a.cpu().numpy(), ref.a) and np.array_equal(L.b.cpu().numpy(), ref.b)
            Lp = ctx.build(rp, col, g.n_vertices, s, dual, sline.SLINE_NO_WEIGHTS, spgemm=True)
            assert torch.equal(Lp.a, L.a) and torch.equal(Lp.b, L.b) and Lp.w is None
    # caller buffers without w
    g = gen.uniform_2000(12)
    rp, col = to_device(g, dev)
    H = sline.Context.csr(rp, col, g.n_vertices)
    ref, _ = oracle.naive(g.row_ptr, g.col, g.n_edges, g.n_vertices, 1)
    buf = torch.zeros(2 * len(ref), dtype=torch.int32, device=dev)
    out = sline.sline_edges(0, len(ref), buf[:len(ref)].data_ptr(), buf[len(ref):].data_ptr(), None)
    assert sline.sline_build(ctx.ctx, H, 1, 0, sline.SLINE_NO_WEIGHTS, out) == sline.SLINE_OK
    assert np.array_equal(buf[:len(ref)].cpu().numpy(), ref.a)
    # without the flag a missing w is an error
    out = sline.sline_edges(0, len(ref), buf[:len(ref)].data_ptr(), buf[len(ref):].data_ptr(), None)
    assert sline.sline_build(ctx.ctx, H, 1, 0, 0, out) == sline.SLINE_EINVAL
