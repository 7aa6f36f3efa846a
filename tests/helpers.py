"""Test helpers: device upload, output digests and checks.

The digest is the order-independent sum, modulo 2^64, of a mixing function of
each output triple (a, b, w).  ``digest_torch`` recomputes, with torch integer
ops on whatever device holds the tensors, the same function the oracle sums in
C (``oracle_mix``); a CPU test pins the two against each other.
"""

from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1


def _s64(x: int) -> int:
    x &= M64
    return x - (1 << 64) if x >= (1 << 63) else x


_C1 = _s64(0x9E3779B97F4A7C15)
_C2 = _s64(0xC2B2AE3D27D4EB4F)
_C3 = _s64(0x165667B19E3779F9)
_C4 = _s64(0xD6E8FEB86659FD93)


def mix_py(a: int, b: int, w: int) -> int:
    """Reference of the digest term in plain Python integers."""
    x = ((a & 0xFFFFFFFF) * 0x9E3779B97F4A7C15) & M64
    x ^= ((b & 0xFFFFFFFF) * 0xC2B2AE3D27D4EB4F) & M64
    x ^= ((w & 0xFFFFFFFF) * 0x165667B19E3779F9) & M64
    x ^= x >> 31
    x = (x * 0xD6E8FEB86659FD93) & M64
    x ^= x >> 32
    return x


def digest_torch(a, b, w, chunk: int = 1 << 26) -> int:
    """Sum of mix(a, b, w) over all entries, mod 2^64 (torch int64 arithmetic)."""
    import torch

    n = int(a.shape[0])
    lo_sum = 0
    hi_sum = 0
    for i in range(0, n, chunk):
        A = a[i:i + chunk].to(torch.int64)
        B = b[i:i + chunk].to(torch.int64)
        W = w[i:i + chunk].to(torch.int64)
        x = (A * _C1) ^ (B * _C2) ^ (W * _C3)
        x = x ^ ((x >> 31) & ((1 << 33) - 1))
        x = x * _C4
        x = x ^ ((x >> 32) & ((1 << 32) - 1))
        lo_sum += int((x & 0xFFFFFFFF).sum().item())
        hi_sum += int(((x >> 32) & 0xFFFFFFFF).sum().item())
        del A, B, W, x
    return (lo_sum + (hi_sum << 32)) & M64


def check_canonical_torch(a, b, w, s: int, chunk: int = 1 << 26) -> None:
    """a < b, w >= s, and (a, b) strictly increasing across the whole array."""
    import torch

    n = int(a.shape[0])
    prev = None
    for i in range(0, n, chunk):
        A = a[i:i + chunk]
        B = b[i:i + chunk]
        W = w[i:i + chunk]
        assert bool((A < B).all()), "a < b violated"
        assert bool((W >= s).all()), "w >= s violated"
        key = A.to(torch.int64) * (1 << 32) + B.to(torch.int64)
        if key.numel() > 1:
            assert bool((key[1:] > key[:-1]).all()), "not sorted by (a, b)"
        if prev is not None and key.numel():
            assert int(key[0].item()) > prev, "not sorted across chunks"
        if key.numel():
            prev = int(key[-1].item())


def row_slice(L, rows):
    """Host copies of the output rows `rows` (ascending) of a device result."""
    import torch

    r = torch.as_tensor(np.asarray(rows, dtype=np.int32), device=L.a.device)
    lo = torch.searchsorted(L.a, r, right=False)
    hi = torch.searchsorted(L.a, r, right=True)
    lo, hi = lo.cpu().numpy(), hi.cpu().numpy()
    parts_a, parts_b, parts_w = [], [], []
    for x, y in zip(lo, hi):
        parts_a.append(L.a[x:y].cpu().numpy())
        parts_b.append(L.b[x:y].cpu().numpy())
        parts_w.append(L.w[x:y].cpu().numpy())
    cat = lambda p: np.concatenate(p) if p else np.zeros(0, np.int32)
    return cat(parts_a), cat(parts_b), cat(parts_w)


def to_device(g, dev):
    import torch

    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int32)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).to(dev)
    return rp, col


def assert_same(L, ref, what: str = "") -> None:
    a, b, w = L.a.cpu().numpy(), L.b.cpu().numpy(), L.w.cpu().numpy()
    assert len(a) == len(ref.a), f"{what}: {len(a)} pairs vs oracle {len(ref.a)}"
    for x, y, name in zip((a, b, w), (ref.a, ref.b, ref.w), "abw"):
        if not np.array_equal(x, y):
            bad = int(np.flatnonzero(x != y)[0])
            raise AssertionError(f"{what}: {name} differs first at {bad}: "
                                 f"got ({a[bad]},{b[bad]},{w[bad]}) want "
                                 f"({ref.a[bad]},{ref.b[bad]},{ref.w[bad]})")
