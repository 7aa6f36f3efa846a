"""Python binding of libsline (include/sline.h) -- argument marshalling only.

Every computation runs in the HIP library ``libsline.so`` built from
``csrc/``; this module only passes pointers and sizes.  If the library is
missing it raises -- there is no CPU fallback.  PyTorch supplies device memory
(through the allocator callbacks of ``sline_allocator``) and the stream.

Low-level names mirror the C-ABI (``sline_create``, ``sline_build``, ...);
``Context`` wraps them for torch tensors.
"""

from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsline.so")

SLINE_OK = 0
SLINE_EINVAL = -1
SLINE_ENOMEM = -2
SLINE_ECAPACITY = -3
SLINE_EDEVICE = -4
SLINE_EBUSY = -5
SLINE_SKIP_VALIDATE = 1
SLINE_PROFILE = 2
SLINE_NO_WEIGHTS = 4
SLINE_REUSE_LOOKAHEAD = 1
SLINE_RELABEL_DESC = 8
SLINE_RELABEL_ASC = 16
SLINE_NO_PRUNE = 32
SLINE_NO_VISITED = 64
SLINE_NO_SHORTCUT = 128
# the variants of Table III as sline_build flags
VARIANT_FLAGS = {"f0": 0, "f1": SLINE_NO_VISITED | SLINE_NO_SHORTCUT,
                 "f2": SLINE_NO_PRUNE | SLINE_NO_SHORTCUT, "f3": SLINE_NO_PRUNE | SLINE_NO_VISITED,
                 "f4": SLINE_NO_PRUNE | SLINE_NO_VISITED | SLINE_NO_SHORTCUT}

_i32p = ctypes.POINTER(ctypes.c_int32)


class sline_csr(ctypes.Structure):
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("n_edges", ctypes.c_int32), ("n_vertices", ctypes.c_int32)]


class sline_edges(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class sline_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("n_items", "nnz", "nnz_kept", "n_kept", "wedges", "n_pairs", "n_small",
                 "n_heavy", "passes")] + [(k, ctypes.c_double) for k in
                ("ms_transpose", "ms_prepare", "ms_count", "ms_scan", "ms_fill")] + [
                (k, ctypes.c_int64) for k in ("heavy_nnz", "heavy_wedges", "heavy_pairs")] + [
                ("ms_tasks", ctypes.c_double), ("product_nnz", ctypes.c_int64),
                ("ms_product", ctypes.c_double), ("ms_filter", ctypes.c_double),
                ("intersections", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: (float(getattr(self, k)) if k.startswith("ms_") else int(getattr(self, k)))
                for k, _ in self._fields_}


class sline_tuning(ctypes.Structure):
    _fields_ = [("small_max_wedges", ctypes.c_int32), ("task_wedges", ctypes.c_int32),
                ("group_parts", ctypes.c_int32), ("light_len", ctypes.c_int32),
                ("small_grid_per_cu", ctypes.c_int32), ("task_grid_per_cu", ctypes.c_int32),
                ("stage_max_bytes", ctypes.c_int64), ("dense_min_wedges", ctypes.c_int32),
                ("small_slots", ctypes.c_int32), ("task_slots", ctypes.c_int32),
                ("tiny_max_wedges", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class sline_graph(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_arcs", ctypes.c_int64),
                ("old_id", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class sline_query_info(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("t_submit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("batch_size", ctypes.c_int32), ("status", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class sline_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class SlineError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_str(status)} ({status}): {message}")
        self.status = status


_lib = None

# name -> (restype, argtypes); every name here is declared in include/sline.h
SIGNATURES = {
    "sline_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                      ctypes.POINTER(sline_allocator)]),
    "sline_destroy": (None, [ctypes.c_void_p]),
    "sline_build": (ctypes.c_int32, [ctypes.c_void_p, sline_csr, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_uint32, ctypes.POINTER(sline_edges)]),
    "sline_build_spgemm": (ctypes.c_int32, [ctypes.c_void_p, sline_csr, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_uint32,
                                            ctypes.POINTER(sline_edges)]),
    "sline_build_noalloc": (ctypes.c_int32, [ctypes.c_void_p, sline_csr, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_uint32,
                                             ctypes.POINTER(sline_edges)]),
    "sline_build_batch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(sline_csr),
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32,
                                           ctypes.POINTER(sline_edges)]),
    "sline_batch_plan_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.POINTER(sline_csr),
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32,
                                                 ctypes.POINTER(ctypes.c_void_p)]),
    "sline_batch_plan_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(sline_edges)]),
    "sline_batch_plan_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "sline_batch_plan_destroy": (None, [ctypes.c_void_p]),
    "sline_edges_free": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_edges)]),
    "sline_filter": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_edges), ctypes.c_int32,
                                      ctypes.c_uint32, ctypes.POINTER(sline_edges)]),
    "sline_build_sweep": (ctypes.c_int32, [ctypes.c_void_p, sline_csr, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                           ctypes.c_uint32, ctypes.POINTER(sline_edges)]),
    "sline_squeeze": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(sline_edges),
                                       ctypes.c_uint32, ctypes.POINTER(sline_graph)]),
    "sline_graph_free": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_graph)]),
    "sline_components": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(sline_edges), ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "sline_last_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_stats)]),
    "sline_get_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_tuning)]),
    "sline_set_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_tuning)]),
    "sline_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "sline_server_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                             ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "sline_server_register": (ctypes.c_int32, [ctypes.c_void_p, sline_csr,
                                               ctypes.POINTER(ctypes.c_int32)]),
    "sline_server_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "sline_server_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(sline_edges),
                                           ctypes.POINTER(sline_query_info)]),
    "sline_server_release": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(sline_edges)]),
    "sline_server_pending": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int32)]),
    "sline_server_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "sline_server_set_reuse": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_uint32]),
    "sline_server_reuse_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                                  ctypes.POINTER(ctypes.c_int64),
                                                  ctypes.POINTER(ctypes.c_int64)]),
    "sline_server_destroy": (None, [ctypes.c_void_p]),
    "sline_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}


def load(path: str | None = None):
    """Load libsline.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libsline is not built ({p} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().sline_status_str(status).decode()


# ------------------------------------------------------- C-ABI mirrors

def sline_create(device: int = 0, hip_stream: int | None = None,
                 allocator: sline_allocator | None = None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    st = load().sline_create(ctypes.byref(ctx), device, hip_stream,
                             ctypes.byref(allocator) if allocator is not None else None)
    if st != SLINE_OK:
        raise SlineError(st, "sline_create failed")
    return ctx


def sline_destroy(ctx) -> None:
    load().sline_destroy(ctx)


def sline_build(ctx, csr: sline_csr, s: int, dual: int, flags: int, out: sline_edges) -> int:
    return load().sline_build(ctx, csr, s, dual, flags, ctypes.byref(out))


def sline_build_noalloc(ctx, csr: sline_csr, s: int, dual: int, flags: int,
                        out: sline_edges) -> int:
    return load().sline_build_noalloc(ctx, csr, s, dual, flags, ctypes.byref(out))


def sline_build_batch(ctx, csrs, s, dual, flags: int, outs) -> int:
    """csrs: sequence of sline_csr; s, dual: int sequences; outs: ctypes array of sline_edges."""
    G = len(csrs)
    carr = (sline_csr * G)(*csrs)
    sarr = (ctypes.c_int32 * G)(*[int(x) for x in s])
    darr = (ctypes.c_int32 * G)(*[int(x) for x in dual])
    return load().sline_build_batch(ctx, G, carr, sarr, darr, flags, outs)


def sline_edges_free(ctx, edges: sline_edges) -> int:
    return load().sline_edges_free(ctx, ctypes.byref(edges))


def sline_last_stats(ctx) -> sline_stats:
    st = sline_stats()
    load().sline_last_stats(ctx, ctypes.byref(st))
    return st


def sline_get_tuning(ctx) -> sline_tuning:
    t = sline_tuning()
    st = load().sline_get_tuning(ctx, ctypes.byref(t))
    if st != SLINE_OK:
        raise SlineError(st, "sline_get_tuning failed")
    return t


def sline_set_tuning(ctx, tuning: sline_tuning) -> int:
    return load().sline_set_tuning(ctx, ctypes.byref(tuning))


def sline_last_error(ctx) -> str:
    return load().sline_last_error(ctx).decode()


def sline_status_str(status: int) -> str:
    return status_str(status)


# --------------------------------------------------------- torch layer

@dataclass
class LineGraph:
    """L_s as device tensors (int32): pairs (a[k], b[k]) with overlap w[k]."""

    a: "object"
    b: "object"
    w: "object"

    def __len__(self) -> int:
        return int(self.a.shape[0])


def torch_allocator(device: int):
    """An sline_allocator backed by PyTorch's caching allocator."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0))
        except Exception:
            return None

    def _free(ptr, nbytes, stream, user):
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    alloc = sline_allocator(fa, ff, None)
    alloc._keep = (fa, ff)  # keep the callbacks alive with the struct
    return alloc


class Context:
    """A libsline context on one device and torch stream."""

    def __init__(self, device: int = 0, stream=None, torch_memory: bool = True):
        import torch
        load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc = torch_allocator(device) if torch_memory else None
        self.ctx = sline_create(device, self.stream.cuda_stream, self._alloc)
        self._plans = weakref.WeakSet()  # open BatchPlans: destroyed before the context

    def close(self) -> None:
        if self.ctx:
            for plan in list(self._plans):
                plan.close()
            sline_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def csr(row_ptr, col, n_vertices: int) -> sline_csr:
        import torch
        for t in (row_ptr, col):
            if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("row_ptr and col must be contiguous int32 device tensors")
        return sline_csr(row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                         int(row_ptr.numel()) - 1, int(n_vertices))

    def build(self, row_ptr, col, n_vertices: int, s: int, dual: int = 0,
              flags: int = 0, spgemm: bool = False) -> LineGraph:
        """L_s(H) (or L_s(H*) with dual=1) as int32 device tensors sorted by (a, b).

        spgemm=True takes the product route (sline_build_spgemm)."""
        import torch
        fn = load().sline_build_spgemm if spgemm else load().sline_build
        H = self.csr(row_ptr, col, n_vertices)
        dev = torch.device("cuda", self.device)
        probe = torch.empty(3, dtype=torch.int32, device=dev)
        out = sline_edges(0, 1, probe[0:1].data_ptr(), probe[1:2].data_ptr(), probe[2:3].data_ptr())
        nw = bool(flags & SLINE_NO_WEIGHTS)
        st = fn(self.ctx, H, s, dual, flags, ctypes.byref(out))
        if st == SLINE_OK:
            n = int(out.n_pairs)  # 0 or 1 pair: it sits in the probe buffers
            return LineGraph(probe[0:n].clone(), probe[1:1 + n].clone(),
                             None if nw else probe[2:2 + n].clone())
        if st != SLINE_ECAPACITY:
            raise SlineError(st, sline_last_error(self.ctx))
        n = int(out.n_pairs)
        a = torch.empty(n, dtype=torch.int32, device=dev)
        b = torch.empty(n, dtype=torch.int32, device=dev)
        w = None if nw else torch.empty(n, dtype=torch.int32, device=dev)
        out = sline_edges(0, n, a.data_ptr(), b.data_ptr(), None if nw else w.data_ptr())
        st = fn(self.ctx, H, s, dual, flags, ctypes.byref(out))
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return LineGraph(a, b, w)

    def build_noalloc(self, row_ptr, col, n_vertices: int, s: int, dual: int = 0,
                      flags: int = 0, a=None, b=None, w=None):
        """sline_build_noalloc into the caller's int32 device tensors a, b, w
        (equal lengths; w may be None with SLINE_NO_WEIGHTS).  Returns
        (status, n_pairs); on SLINE_OK the first n_pairs entries hold L_s."""
        cap = int(a.numel())
        out = sline_edges(0, cap, a.data_ptr(), b.data_ptr(),
                          None if w is None else w.data_ptr())
        st = sline_build_noalloc(self.ctx, self.csr(row_ptr, col, n_vertices), s, dual, flags,
                                 out)
        return st, int(out.n_pairs)

    def build_owned(self, row_ptr, col, n_vertices: int, s: int, dual: int = 0,
                    flags: int = 0) -> sline_edges:
        """One sline_build call whose output the library allocates (capacity 0);
        release it with ``free_edges([out])``."""
        out = sline_edges()
        st = sline_build(self.ctx, self.csr(row_ptr, col, n_vertices), s, dual, flags, out)
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return out

    def _tuned(self, tuning_cache, graphs, s, dual):
        """The tuning cached for this batch's class, applied around a call."""
        from . import autotune
        if tuning_cache is None:
            return autotune.cached_tuning(self, None, "")
        return autotune.cached_tuning(self, tuning_cache,
                                      autotune.batch_signature(graphs, s, dual))

    def build_batch_owned(self, graphs, s, dual=None, flags: int = 0,
                          tuning_cache: str | None = None):
        """One sline_build_batch call whose outputs the library allocates
        (capacity 0): returns the ``sline_edges`` array; release every entry
        with ``free_edges``.  ``tuning_cache``: an autotuner cache file whose
        entry for this batch's class applies to the call."""
        G = len(graphs)
        dual = [0] * G if dual is None else list(dual)
        csrs = [self.csr(rp, col, n) for rp, col, n in graphs]
        outs = (sline_edges * max(G, 1))()
        with self._tuned(tuning_cache, graphs, s, dual):
            st = sline_build_batch(self.ctx, csrs, s, dual, flags, outs)
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return outs

    def free_edges(self, outs, n: int | None = None) -> None:
        for g in range(len(outs) if n is None else n):
            sline_edges_free(self.ctx, outs[g])

    def build_batch(self, graphs, s, dual=None, flags: int = 0,
                    library_alloc: bool = False,
                    tuning_cache: str | None = None) -> list[LineGraph]:
        """L_{s[g]} of every graph (row_ptr, col, n_vertices) in one batched call.

        library_alloc=True lets the library allocate the outputs (the results
        are copied into torch tensors and the library's arrays released).
        tuning_cache: an autotuner cache file whose entry for this batch's
        class applies to the call."""
        import torch
        G = len(graphs)
        if library_alloc:
            outs = self.build_batch_owned(graphs, s, dual, flags, tuning_cache)
            dev = torch.device("cuda", self.device)
            nw = bool(flags & SLINE_NO_WEIGHTS)

            def col(ptr, n, weights):
                if weights and nw:
                    return None
                if n == 0 or not ptr:
                    return torch.empty(0, dtype=torch.int32, device=dev)
                return torch.as_tensor(_DeviceArray(ptr, n), device=dev).clone()

            res = []
            for g in range(G):
                n = int(outs[g].n_pairs)
                res.append(LineGraph(col(outs[g].a, n, False), col(outs[g].b, n, False),
                                     col(outs[g].w, n, True)))
            torch.cuda.synchronize(dev)
            self.free_edges(outs, G)
            return res
        dual = [0] * G if dual is None else list(dual)
        csrs = [self.csr(rp, col, n) for rp, col, n in graphs]
        dev = torch.device("cuda", self.device)
        probe = torch.empty((3, max(G, 1)), dtype=torch.int32, device=dev)
        outs = (sline_edges * max(G, 1))()
        for g in range(G):
            outs[g] = sline_edges(0, 1, probe[0, g:].data_ptr(), probe[1, g:].data_ptr(),
                                  probe[2, g:].data_ptr())
        with self._tuned(tuning_cache, graphs, s, dual):
            st = sline_build_batch(self.ctx, csrs, s, dual, flags, outs)
        if st == SLINE_OK:
            return [LineGraph(probe[0, g:g + int(outs[g].n_pairs)].clone(),
                              probe[1, g:g + int(outs[g].n_pairs)].clone(),
                              probe[2, g:g + int(outs[g].n_pairs)].clone()) for g in range(G)]
        if st != SLINE_ECAPACITY:
            raise SlineError(st, sline_last_error(self.ctx))
        need = [int(outs[g].n_pairs) for g in range(G)]
        bufs = []
        for g in range(G):
            t = torch.empty((3, max(need[g], 1)), dtype=torch.int32, device=dev)
            bufs.append(t)
            outs[g] = sline_edges(0, max(need[g], 1), t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr())
        with self._tuned(tuning_cache, graphs, s, dual):
            st = sline_build_batch(self.ctx, csrs, s, dual, flags, outs)
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return [LineGraph(bufs[g][0, :need[g]], bufs[g][1, :need[g]], bufs[g][2, :need[g]])
                for g in range(G)]

    # ------------------------------------------------ after L_s (Table I)

    @staticmethod
    def edges_of(L: "LineGraph") -> sline_edges:
        """An sline_edges view (capacity 0) of a LineGraph's device tensors."""
        n = len(L)
        ptr = lambda t: (t.data_ptr() if (t is not None and t.numel()) else None)
        return sline_edges(n, 0, ptr(L.a), ptr(L.b), ptr(L.w))

    def _take(self, out: sline_edges, weights: bool = True) -> LineGraph:
        """Copy a library-allocated result into torch tensors and free it."""
        import torch
        dev = torch.device("cuda", self.device)
        n = int(out.n_pairs)

        def col(ptr):
            if n == 0 or not ptr:
                return torch.empty(0, dtype=torch.int32, device=dev)
            return torch.as_tensor(_DeviceArray(ptr, n), device=dev).clone()

        L = LineGraph(col(out.a), col(out.b), col(out.w) if weights else None)
        torch.cuda.synchronize(dev)
        sline_edges_free(self.ctx, out)
        return L

    def filter(self, L: LineGraph, s: int, flags: int = 0) -> LineGraph:
        """L_s from a weighted L_s' (s' <= s): sline_filter."""
        src = self.edges_of(L)
        out = sline_edges()
        st = load().sline_filter(self.ctx, ctypes.byref(src), s, flags, ctypes.byref(out))
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return self._take(out, not (flags & SLINE_NO_WEIGHTS))

    def build_sweep(self, row_ptr, col, n_vertices: int, s_list, dual: int = 0,
                    flags: int = 0) -> list[LineGraph]:
        """L_s for every s of s_list, only the smallest counted (sline_build_sweep)."""
        n = len(s_list)
        outs = (sline_edges * max(n, 1))()
        sarr = (ctypes.c_int32 * max(n, 1))(*[int(x) for x in s_list])
        st = load().sline_build_sweep(self.ctx, self.csr(row_ptr, col, n_vertices), n, sarr, dual,
                                      flags, outs)
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return [self._take(outs[i]) for i in range(n)]

    def squeeze(self, L: LineGraph, n_items: int, flags: int = 0) -> dict:
        """ID squeezing and the symmetric adjacency (sline_squeeze), as torch tensors."""
        import torch
        src = self.edges_of(L)
        g = sline_graph()
        st = load().sline_squeeze(self.ctx, n_items, ctypes.byref(src), flags, ctypes.byref(g))
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        dev = torch.device("cuda", self.device)

        def view(ptr, n, typestr, dtype):
            if n == 0 or not ptr:
                return torch.empty(0, dtype=dtype, device=dev)
            return torch.as_tensor(_DeviceArray(ptr, n, typestr), device=dev).clone()

        out = {"n_nodes": int(g.n_nodes), "n_arcs": int(g.n_arcs),
               "old_id": view(g.old_id, g.n_nodes, "<i4", torch.int32),
               "row_ptr": view(g.row_ptr, g.n_nodes + 1, "<i8", torch.int64),
               "col": view(g.col, g.n_arcs, "<i4", torch.int32),
               "w": None if flags & SLINE_NO_WEIGHTS else view(g.w, g.n_arcs, "<i4", torch.int32)}
        torch.cuda.synchronize(dev)
        load().sline_graph_free(self.ctx, ctypes.byref(g))
        return out

    def components(self, L: LineGraph, n_items: int):
        """s-connected components (sline_components): (comp tensor, count)."""
        import torch
        comp = torch.empty(max(n_items, 1), dtype=torch.int32, device=torch.device("cuda", self.device))
        src = self.edges_of(L)
        cnt = ctypes.c_int64()
        st = load().sline_components(self.ctx, n_items, ctypes.byref(src), comp.data_ptr(),
                                     ctypes.byref(cnt))
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))
        return comp[:n_items], int(cnt.value)

    def stats(self) -> dict:
        return sline_last_stats(self.ctx).as_dict()

    def tuning(self) -> dict:
        return sline_get_tuning(self.ctx).as_dict()

    def set_tuning(self, **kw) -> None:
        t = sline_get_tuning(self.ctx)
        for k, v in kw.items():
            if not hasattr(t, k):
                raise KeyError(k)
            setattr(t, k, int(v))
        st = sline_set_tuning(self.ctx, t)
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx))


# -------------------------------------------------------------- serving

class BatchPlan:
    """A batch sized once and replayed as one HIP graph launch
    (sline_batch_plan_* of the C-ABI).

    ``graphs`` are (row_ptr, col, n_vertices) int32 device tensors; they are
    kept alive with the plan and may be changed in place between runs (same
    row_ptr[-1]).  ``tuning_cache``: an autotuner cache file whose entry for
    this batch's class the plan is made with.  ``run`` returns each graph's L_s as views into the plan's
    result arrays (valid until the next run or ``close``), or copies."""

    def __init__(self, ctx: "Context", graphs, s, dual=None, flags: int = 0,
                 tuning_cache: str | None = None):
        G = len(graphs)
        self.ctx = ctx
        self.G = G
        self.flags = flags
        self._graphs = list(graphs)
        dual = [0] * G if dual is None else list(dual)
        carr = (sline_csr * max(G, 1))(*[Context.csr(rp, col, n) for rp, col, n in graphs])
        sarr = (ctypes.c_int32 * max(G, 1))(*[int(x) for x in s])
        darr = (ctypes.c_int32 * max(G, 1))(*[int(x) for x in dual])
        self.plan = ctypes.c_void_p()
        # the plan keeps the tuning it was created with
        with ctx._tuned(tuning_cache, graphs, s, dual):
            st = load().sline_batch_plan_create(ctx.ctx, G, carr, sarr, darr, flags,
                                                ctypes.byref(self.plan))
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(ctx.ctx))
        self._outs = (sline_edges * max(G, 1))()
        ctx._plans.add(self)

    def info(self) -> tuple[int, int, int]:
        """(device bytes held, task capacity, pair capacity)."""
        b, t, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        st = load().sline_batch_plan_info(self.plan, ctypes.byref(b), ctypes.byref(t),
                                          ctypes.byref(p))
        if st != SLINE_OK:
            raise SlineError(st, "sline_batch_plan_info failed")
        return int(b.value), int(t.value), int(p.value)

    def run_raw(self, s=None) -> int:
        """One replay; returns the status (results in ``self._outs``)."""
        if not self.plan:
            raise RuntimeError("the batch plan is closed (or its context is)")
        sarr = None
        if s is not None:
            if len(s) != self.G:
                raise ValueError(f"{len(s)} values of s for {self.G} graphs")
            sarr = (ctypes.c_int32 * max(self.G, 1))(*[int(x) for x in s])
        return load().sline_batch_plan_run(self.plan, sarr, self._outs)

    def run(self, s=None, copy: bool = False) -> list[LineGraph]:
        import torch
        st = self.run_raw(s)
        if st != SLINE_OK:
            raise SlineError(st, sline_last_error(self.ctx.ctx))
        dev = torch.device("cuda", self.ctx.device)

        def col(ptr, n):
            if not ptr or n == 0:
                return torch.empty(0, dtype=torch.int32, device=dev)
            t = torch.as_tensor(_DeviceArray(ptr, n), device=dev)
            return t.clone() if copy else t

        res = []
        for g in range(self.G):
            o = self._outs[g]
            n = int(o.n_pairs)
            w = None if (self.flags & SLINE_NO_WEIGHTS) else col(o.w, n)
            res.append(LineGraph(col(o.a, n), col(o.b, n), w))
        return res

    def close(self) -> None:
        if self.plan:
            load().sline_batch_plan_destroy(self.plan)
            self.plan = None
            self.ctx._plans.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Zero-copy view of a device array (int32 by default) for torch.as_tensor."""

    def __init__(self, ptr: int, n: int, typestr: str = "<i4"):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}


class Server:
    """A query loop over registered hypergraphs (sline_server_* of the C-ABI)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 64 << 30, max_batch: int = 64,
                 workers: int = 2):
        lib = load()
        self.device = device
        self.srv = ctypes.c_void_p()
        st = lib.sline_server_create(ctypes.byref(self.srv), device, int(hbm_budget_bytes),
                                     int(max_batch), int(workers))
        if st != SLINE_OK:
            raise SlineError(st, "sline_server_create failed")
        self._keep = []

    def register(self, row_ptr, col, n_vertices: int) -> int:
        gid = ctypes.c_int32()
        st = load().sline_server_register(self.srv, Context.csr(row_ptr, col, n_vertices),
                                          ctypes.byref(gid))
        if st != SLINE_OK:
            raise SlineError(st, "sline_server_register failed")
        self._keep.append((row_ptr, col))
        return int(gid.value)

    def submit(self, graph_id: int, s: int, dual: int = 0) -> int:
        t = ctypes.c_int64()
        st = load().sline_server_submit(self.srv, graph_id, s, dual, ctypes.byref(t))
        if st != SLINE_OK:
            raise SlineError(st, "sline_server_submit failed")
        return int(t.value)

    def set_reuse(self, cache_bytes: int, min_nnz: int = 0, lookahead: bool = False) -> None:
        """Result reuse (sline_server_set_reuse); cache_bytes = 0 turns it off;
        lookahead sets SLINE_REUSE_LOOKAHEAD."""
        st = load().sline_server_set_reuse(self.srv, int(cache_bytes), int(min_nnz),
                                           SLINE_REUSE_LOOKAHEAD if lookahead else 0)
        if st != SLINE_OK:
            raise SlineError(st, "sline_server_set_reuse failed")

    def reuse_stats(self) -> dict:
        r, k, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        load().sline_server_reuse_stats(self.srv, ctypes.byref(r), ctypes.byref(k), ctypes.byref(b))
        return {"reused": int(r.value), "kept": int(k.value), "kept_bytes": int(b.value)}

    def pending(self) -> tuple[int, int]:
        q, r = ctypes.c_int64(), ctypes.c_int32()
        load().sline_server_pending(self.srv, ctypes.byref(q), ctypes.byref(r))
        return int(q.value), int(r.value)

    def poll(self, ticket: int, keep: bool = True):
        """None while running; else (LineGraph copy or None, info dict)."""
        import torch
        out = sline_edges()
        info = sline_query_info()
        st = load().sline_server_poll(self.srv, ticket, ctypes.byref(out), ctypes.byref(info))
        if st == SLINE_EBUSY:
            return None
        if st != SLINE_OK:
            raise SlineError(st, load().sline_server_last_error(self.srv).decode())
        n = int(out.n_pairs)
        L = None
        if keep:
            dev = torch.device("cuda", self.device)
            if n > 0:
                L = LineGraph(*[torch.as_tensor(_DeviceArray(p, n), device=dev).clone()
                                for p in (out.a, out.b, out.w)])
            else:
                L = LineGraph(*[torch.empty(0, dtype=torch.int32, device=dev) for _ in range(3)])
            torch.cuda.synchronize(dev)
        load().sline_server_release(self.srv, ctypes.byref(out))
        return L, info.as_dict()

    def close(self) -> None:
        if self.srv:
            load().sline_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
