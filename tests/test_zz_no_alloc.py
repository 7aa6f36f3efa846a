"""sline_build_noalloc: the allocation-free variant of sline_build.

Called through the C-ABI with caller buffers; every result must equal
sline_build's on the same input (and the oracle's), bit for bit.  Two calls in
a row, the second on a smaller input, check that the shared scratch array
keeps no state that leaks from one call into the next; calls of the plain
entry point in between check that the context's own workspace is left as it
was.  Inputs beyond the scratch array are refused with SLINE_ENOMEM before
any counting kernel runs.
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


def _noalloc(ctx, g, dev, s, dual, cap=None, flags=0):
    """One sline_build_noalloc call into fresh caller buffers."""
    import torch
    from paper_2010_11448_amd import sline

    rp, col = to_device(g, dev)
    if cap is None:
        # room for the result: the plain build says how much
        cap = max(1, len(ctx.build(rp, col, g.n_vertices, s, dual)))
    a = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    b = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    w = None if flags & sline.SLINE_NO_WEIGHTS else torch.full((cap,), -7, dtype=torch.int32,
                                                               device=dev)
    st, n = ctx.build_noalloc(rp, col, g.n_vertices, s, dual, flags, a, b, w)
    return st, n, a, b, w


def _check_against_plain(ctx, g, dev, s, dual, what):
    from paper_2010_11448_amd import sline

    print(f"case: noalloc {what} s={s} dual={dual}", flush=True)
    rp, col = to_device(g, dev)
    plain = ctx.build(rp, col, g.n_vertices, s, dual)
    st, n, a, b, w = _noalloc(ctx, g, dev, s, dual, cap=max(1, len(plain)) + 5)
    assert st == sline.SLINE_OK, sline.sline_last_error(ctx.ctx)
    assert n == len(plain), f"{what}: {n} pairs vs plain {len(plain)}"
    for got, want, name in ((a, plain.a, "a"), (b, plain.b, "b"), (w, plain.w, "w")):
        assert np.array_equal(got[:n].cpu().numpy(), want.cpu().numpy()), f"{what}: {name}"
    # nothing written past the result
    assert bool((a[n:] == -7).all()) and bool((b[n:] == -7).all()) and bool((w[n:] == -7).all())
    return n, a, b, w


@pytest.mark.parametrize("dual", [0, 1])
def test_two_calls_second_smaller(ctx, dual):
    """A larger input, then a smaller one, through the no-allocation entry point."""
    import torch
    from paper_2010_11448_amd import sline

    dev = torch.device("cuda", 0)
    big = gen.batch_graph(5).graph            # a batch-law graph, tens of thousands of items
    small = gen.uniform_2000(12)
    for g, s, what in ((big, 2, "batch-law graph 5"), (small, 1, "uniform 2000x5000 seed 12")):
        n, a, b, w = _check_against_plain(ctx, g, dev, s, dual, what)
        ref, _ = oracle.wedge(g.row_ptr, g.col, g.n_edges, g.n_vertices, s, dual=dual, threads=8)
        assert_same(sline.LineGraph(a[:n], b[:n], w[:n]), ref, f"noalloc {what} vs oracle")


def test_interleaved_with_plain_builds(ctx):
    """No-allocation calls between plain calls on one context, both sides, several s."""
    import torch

    dev = torch.device("cuda", 0)
    graphs = [gen.uniform_2000(11), gen.batch_graph(7).graph, gen.random_small(300, 200, 12, 5),
              gen.nested_chain(30, 4, seed=3)]
    for i, g in enumerate(graphs):
        for s in (1, 3):
            for dual in (0, 1):
                _check_against_plain(ctx, g, dev, s, dual, f"graph {i}")


def test_no_weights_and_capacity(ctx):
    """SLINE_NO_WEIGHTS writes a and b only; too small a buffer reports the need."""
    import torch
    from paper_2010_11448_amd import sline

    dev = torch.device("cuda", 0)
    g = gen.uniform_2000(13)
    rp, col = to_device(g, dev)
    plain = ctx.build(rp, col, g.n_vertices, 2, 0)
    need = len(plain)
    assert need > 10
    st, n, a, b, w = _noalloc(ctx, g, dev, 2, 0, cap=need - 1)
    assert st == sline.SLINE_ECAPACITY and n == need
    assert bool((a == -7).all()) and bool((b == -7).all()) and bool((w == -7).all())
    st, n, a, b, w = _noalloc(ctx, g, dev, 2, 0, cap=need, flags=sline.SLINE_NO_WEIGHTS)
    assert st == sline.SLINE_OK and n == need and w is None
    assert np.array_equal(a.cpu().numpy(), plain.a.cpu().numpy())
    assert np.array_equal(b.cpu().numpy(), plain.b.cpu().numpy())


def test_refusals(ctx):
    """Library-allocated output is refused; so is an input beyond the scratch array."""
    import torch
    from paper_2010_11448_amd import sline

    dev = torch.device("cuda", 0)
    g = gen.uniform_2000(11)
    rp, col = to_device(g, dev)
    out = sline.sline_edges()  # capacity 0: the library would have to allocate
    assert sline.sline_build_noalloc(ctx.ctx, ctx.csr(rp, col, g.n_vertices), 1, 0, 0,
                                     out) == sline.SLINE_EINVAL
    # about 4.4 million incidences: its workspace alone is larger than the scratch
    huge = gen.uniform_hypergraph(400_000, 800_000, 2, 20, seed=9)
    assert huge.nnz > 4_000_000
    st, n, a, b, w = _noalloc(ctx, huge, dev, 4, 0, cap=16)
    assert st == sline.SLINE_ENOMEM
    assert "scratch" in sline.sline_last_error(ctx.ctx)
    # the context still works for both entry points afterwards
    _check_against_plain(ctx, g, dev, 2, 1, "after a refusal")
