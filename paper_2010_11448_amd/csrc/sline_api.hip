// Host side of libsline: the C-ABI entry points of include/sline.h, the
// context (stream, allocator, workspace) and the order of the device stages.
//
// sline_build, stage by stage (every stage is a HIP kernel of this library):
//   1. row_ptr check, nnz read-back                      (one host sync)
//   2. row ids, member range / order checks
//   3. transpose: a stable radix sort of the (member, incidence) pairs,
//      whose last pass writes the row ids and the position maps; the member
//      checks are read back                              (one host sync)
//   4. items / member lists chosen by the dual flag (H* swaps the roles, Sec. III)
//   5. s-filtered member lists N_s(v) (degree-based pruning, Sec. IV-C) and
//      the back-pointer of every incidence of a kept item
//   6. exact per-item wedge counts W_a, lookup-only members (s > 1), tasks
//      (one-wave items and workgroup task groups)       (one host sync)
//   7. one counting pass staging each range's pairs, exclusive scan of pairs
//      per task                                          (one host sync)
//   8. output allocation, staged ranges copied to their offsets, tasks
//      without room counted again                      (one host sync)
// sline_build_batch runs the same stages once over many graphs (their items
// numbered one after the other, each with its own s); with library-allocated
// results, stage 8 writes every graph's pairs into that graph's own arrays.
// sline_build_spgemm runs them in product mode and filters the product.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sline.h"
#include "sline_internal.h"

using namespace sl;

// Device scratch of sline_build_noalloc: the whole workspace of one build
// (CSR checks, transpose, filtered lists, task arrays, staging pool), so that
// the entry point never allocates.  Each device holds its own copy from the
// moment the library's code object is loaded on it until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host it only
// names the symbol): it uses the device address taken once per device by
// scratch_address().
static __device__ __align__(256) unsigned char scratch[SLINE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (sline_create calls this).  Null if the lookup failed.
void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        } else {
            g_scratch_ptr[device] = p;
        }
    }
    return g_scratch_ptr[device];
}

}  // namespace

struct sline_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    sline_allocator alloc{};
    bool has_alloc = false;
    int n_cu = 256;
    std::string last_error;
    sline_stats stats{};
    Tuning tune;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *ws2 = nullptr;  // task arrays
    size_t ws2_bytes = 0;
    int64_t *host = nullptr;  // pinned read-back area (64 int64)

    // counting work kept after SLINE_ECAPACITY for an immediate retry
    struct Pending {
        bool valid = false;
        sline_csr H{};
        int32_t s = 0, dual = 0;
        uint32_t flags = 0;
        int64_t total = 0;
    } pending;
    // device views into the workspace kept for the fill pass
    CountArgs fill_args{};
    int64_t fill_total = 0;
    int32_t fill_records = 0;   // staged ranges to copy (stage mode)
    int32_t fill_need = 0;      // tasks to recompute (-1: all, count mode)
    void *pool = nullptr;       // staging pool of the last build
    size_t pool_bytes = 0;
    // stage events (SLINE_PROFILE)
    hipEvent_t ev[8] = {};
    bool profile = false;
    bool no_weights = false;  // SLINE_NO_WEIGHTS of the current build
    // batch result kept after SLINE_ECAPACITY for an immediate retry
    struct BatchPending {
        bool valid = false;
        std::vector<sline_csr> H;
        std::vector<int32_t> s, dual;
        uint32_t flags = 0;
        sline_edges comb{};          // combined result (library-owned)
        std::vector<int64_t> off;    // first pair of each graph, n_graphs + 1
        void *bws = nullptr;         // batch workspace (descriptors, item bases)
        size_t bws_bytes = 0;
        int64_t *ibase_dev = nullptr, *off_dev = nullptr;
    } bpend;
    // a batch whose outputs the library allocates: the fill writes each
    // graph's pairs straight into its own arrays (G > 0 while such a batch runs)
    struct Direct {
        int32_t G = 0;
        sline_edges *outs = nullptr;
        bool done = false;  // the fill handed the outputs over
    } direct;
    // sline_build_noalloc: while `base` is set, the workspace, the task arrays
    // and the staging pool are carved from this fixed device region (the
    // device's scratch array) instead of being allocated; `used` is the end
    // of what the current build has taken.
    struct Fixed {
        char *base = nullptr;
        size_t size = 0;
        size_t used = 0;
    } fixed;
    bool pool_fixed = false;  // c->pool lies in the fixed region: never freed
};

namespace {

struct Fail {
    sline_status st;
};

void set_err(sline_ctx *c, const char *fmt, const char *detail = nullptr) {
    char buf[512];
    snprintf(buf, sizeof buf, fmt, detail ? detail : "");
    c->last_error = buf;
}

void hip_check(sline_ctx *c, hipError_t e, const char *where) {
    if (e == hipSuccess) return;
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    c->last_error = buf;
    throw Fail{SLINE_EDEVICE};
}

void *dev_alloc(sline_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->has_alloc) {
        p = c->alloc.alloc(bytes, (void *)c->stream, c->alloc.user);
    } else {
        if (hipMallocAsync(&p, bytes, c->stream) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    return p;
}

void dev_free(sline_ctx *c, void *p, size_t bytes) {
    if (!p) return;
    if (c->has_alloc) c->alloc.free(p, bytes, (void *)c->stream, c->alloc.user);
    else (void)hipFreeAsync(p, c->stream);
}

// Bump allocator over the context workspace.
struct Arena {
    size_t off = 0;
    char *base = nullptr;
    template <typename T>
    T *take(int64_t n) {
        off = (off + 255) & ~(size_t)255;
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += (size_t)std::max<int64_t>(n, 1) * sizeof(T);
        return p;
    }
};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Fixed-region mode: the next `bytes` of the region, or SLINE_ENOMEM with the
// size the build needs when the region is too small.
char *fixed_take(sline_ctx *c, size_t from, size_t bytes, const char *what) {
    const size_t at = align256(from);
    if (at + bytes > c->fixed.size) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "sline_build_noalloc: %s needs %zu bytes of scratch at offset %zu; "
                 "the scratch holds %zu bytes",
                 what, bytes, at, c->fixed.size);
        c->last_error = buf;
        throw Fail{SLINE_ENOMEM};
    }
    c->fixed.used = at + bytes;
    return c->fixed.base + at;
}

void ensure_ws(sline_ctx *c, size_t bytes) {
    if (c->fixed.base) {
        // the workspace starts the region; the task arrays and the pool follow it
        c->ws = fixed_take(c, 0, bytes, "the workspace");
        c->ws_bytes = bytes;
        return;
    }
    if (c->ws_bytes >= bytes) return;
    if (c->ws) {
        hip_check(c, hipStreamSynchronize(c->stream), "workspace release");
        dev_free(c, c->ws, c->ws_bytes);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    c->ws = dev_alloc(c, want);
    if (!c->ws) {
        set_err(c, "workspace allocation of %s bytes failed", std::to_string(want).c_str());
        throw Fail{SLINE_ENOMEM};
    }
    c->ws_bytes = want;
}

void sync(sline_ctx *c, const char *where) { hip_check(c, hipStreamSynchronize(c->stream), where); }

void release_pool(sline_ctx *c) {
    if (c->pool_fixed) {
        // a pool inside the fixed region is not the allocator's to free
        c->pool = nullptr;
        c->pool_bytes = 0;
        c->pool_fixed = false;
        return;
    }
    if (!c->pool) return;
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, c->pool, c->pool_bytes);
    c->pool = nullptr;
    c->pool_bytes = 0;
}

// Staging pool for `want` pairs (`pair_bytes` each: 8 with weights, 4
// without), halving on failure; returns the pairs it holds (0: none, count
// the pairs in a separate pass instead).
int64_t acquire_pool(sline_ctx *c, int64_t want, int64_t pair_bytes) {
    release_pool(c);
    int64_t cap = std::min<int64_t>(want, c->tune.stage_max_bytes / pair_bytes);
    if (c->fixed.base) {
        // whatever the fixed region has left after the task arrays (tasks
        // that find no room are counted again in the fill pass)
        const size_t at = align256(c->fixed.used);
        const int64_t room = at < c->fixed.size ? (int64_t)((c->fixed.size - at) / pair_bytes) : 0;
        cap = std::min<int64_t>(cap, room);
        if (cap < 256) return 0;
        c->pool = c->fixed.base + at;
        c->pool_bytes = (size_t)(cap * pair_bytes);
        c->pool_fixed = true;
        c->fixed.used = at + c->pool_bytes;
        return cap;
    }
    while (cap >= (1 << 20)) {
        void *p = dev_alloc(c, (size_t)(cap * pair_bytes));
        if (p) {
            c->pool = p;
            c->pool_bytes = (size_t)(cap * pair_bytes);
            return cap;
        }
        cap /= 2;
    }
    if (cap > 0) {
        void *p = dev_alloc(c, (size_t)(cap * pair_bytes));
        if (p) {
            c->pool = p;
            c->pool_bytes = (size_t)(cap * pair_bytes);
            return cap;
        }
    }
    return 0;
}

// Stage marks: 0 start, 1 after transpose, 2 after prepare, 3 after count,
// 4 after scan, 5 before fill, 6 after fill.
void mark(sline_ctx *c, int i) {
    if (c->profile) hip_check(c, hipEventRecord(c->ev[i], c->stream), "event record");
}

double span_ms(sline_ctx *c, int i, int j) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[i], c->ev[j]) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0;
    }
    return ms;
}

struct Layout {
    int32_t *err, *queue, *tcounts;
    int64_t *totals, *passes;
    int32_t *rowid, *ptrT, *colT;
    int32_t *rsK0, *rsK1, *rsV0, *rsV1, *rsHist;  // transpose (radix sort) buffers
    int32_t *kT = nullptr, *posT = nullptr;  // transposed position <-> incidence
    int32_t *ptrS, *itmS;
    int32_t *pos;   // s filter: kept entries before each member-list entry (nnz + 1)
    int32_t *xcol;  // batches: columns of the dual graphs' rows (XD)
    int64_t *cost, *tbase, *part64;
    int32_t *part32, *ntask, *start;
};

// The tuning one build runs with: one lane per tiny item pays off only when
// the items outnumber the lanes of the resident one-wave workgroups several
// times over (a lane walks its item's lists one entry after another).
constexpr int64_t kTinyMinItems = 1 << 15;
Tuning build_tuning(const Tuning &t, int64_t n_items) {
    Tuning u = t;
    if (n_items < kTinyMinItems) u.tiny_max_wedges = 0;
    return u;
}

Layout plan_layout(Arena &A, int64_t m, int64_t n, int64_t nnz, int64_t N, int64_t M, bool filt) {
    Layout L{};
    L.err = A.take<int32_t>(4);
    L.queue = A.take<int32_t>(4);
    L.tcounts = A.take<int32_t>(4);
    L.totals = A.take<int64_t>(4);
    L.passes = A.take<int64_t>(4);
    L.rowid = A.take<int32_t>(nnz);
    L.ptrT = A.take<int32_t>(n + 1);
    L.colT = A.take<int32_t>(nnz);
    L.kT = A.take<int32_t>(nnz);
    L.posT = A.take<int32_t>(nnz);
    L.rsK0 = A.take<int32_t>(nnz);
    L.rsK1 = A.take<int32_t>(nnz);
    L.rsV0 = A.take<int32_t>(nnz);
    L.rsV1 = A.take<int32_t>(nnz);
    L.rsHist = A.take<int32_t>(transpose_hist(nnz));
    const int64_t pmax = scan_partials(std::max<int64_t>({n, N, M, m, nnz}) + 1);
    L.part32 = A.take<int32_t>(pmax);
    L.part64 = A.take<int64_t>(pmax);
    if (filt) {
        L.ptrS = A.take<int32_t>(M + 1);
        L.pos = A.take<int32_t>(nnz + 1);
        L.itmS = A.take<int32_t>(nnz);
    }
    L.cost = A.take<int64_t>(N);
    L.ntask = A.take<int32_t>(N);
    L.tbase = A.take<int64_t>(N + 1);
    L.start = A.take<int32_t>(nnz);
    return L;
}

// Task arrays, sized once the task count is known.
struct TaskLayout {
    int32_t *item, *part, *small, *small_item, *tiny, *tiny_item, *big, *cnt, *need, *ctrs;
    int64_t *off, *part64;
    unsigned long long *pool_head;
    StageRec *log;
    int32_t log_cap;
};

TaskLayout plan_tasks(Arena &A, int64_t T) {
    TaskLayout L{};
    L.log_cap = (int32_t)std::min<int64_t>(INT32_MAX - 1, 2 * T + 65536);
    L.pool_head = A.take<unsigned long long>(1);
    L.ctrs = A.take<int32_t>(4);  // [0] log head, [1] tasks flagged
    L.log = A.take<StageRec>(L.log_cap);
    L.need = A.take<int32_t>(T);
    L.item = A.take<int32_t>(T);
    L.part = A.take<int32_t>(T);
    L.small = A.take<int32_t>(T);
    L.small_item = A.take<int32_t>(T);
    L.tiny = A.take<int32_t>(T);
    L.tiny_item = A.take<int32_t>(T);
    L.big = A.take<int32_t>(T);
    L.cnt = A.take<int32_t>(T);
    L.off = A.take<int64_t>(T + 1);
    L.part64 = A.take<int64_t>(scan_partials(T + 1));
    return L;
}

void ensure_ws2(sline_ctx *c, size_t bytes) {
    if (c->fixed.base) {
        c->ws2 = fixed_take(c, c->ws_bytes, bytes, "the task arrays");
        c->ws2_bytes = bytes;
        return;
    }
    if (c->ws2_bytes >= bytes) return;
    if (c->ws2) {
        hip_check(c, hipStreamSynchronize(c->stream), "workspace release");
        dev_free(c, c->ws2, c->ws2_bytes);
        c->ws2 = nullptr;
        c->ws2_bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    c->ws2 = dev_alloc(c, want);
    if (!c->ws2) {
        set_err(c, "task workspace allocation of %s bytes failed", std::to_string(want).c_str());
        throw Fail{SLINE_ENOMEM};
    }
    c->ws2_bytes = want;
}

void transpose(sline_ctx *c, const Layout &L, const int32_t *col, int32_t n, int64_t nnz) {
    int32_t *const rk[2] = {L.rsK0, L.rsK1};
    int32_t *const rv[2] = {L.rsV0, L.rsV1};
    hip_check(c, launch_transpose(c->stream, col, nnz, n, L.rowid, rk, rv, L.rsHist, L.part32,
                                  L.ptrT, L.colT, L.kT, L.posT),
              "transpose");
}

bool same_call(const sline_ctx::Pending &p, const sline_csr &H, int32_t s, int32_t dual,
               uint32_t flags) {
    return p.valid && p.H.row_ptr == H.row_ptr && p.H.col_idx == H.col_idx &&
           p.H.n_edges == H.n_edges && p.H.n_vertices == H.n_vertices && p.s == s &&
           p.dual == dual && p.flags == flags;
}

// Launch the fill of a counted build into the outputs set in F (stage copy,
// or the counting kernels in fill mode) and wait for it.
void fill_into(sline_ctx *c, CountArgs F) {
    mark(c, 5);
    if (c->fill_need >= 0) {
        // stage mode: move the staged ranges, recompute tasks that found no room
        hip_check(c, launch_stage_copy(c->stream, F, c->fill_records), "stage copy");
        if (c->fill_need > 0) {
            F.mode = kModeFill;
            hip_check(c, launch_count(c->stream, F), "fill pass (recompute)");
        }
    } else {
        F.mode = kModeFill;
        F.need = nullptr;
        hip_check(c, launch_count(c->stream, F), "fill pass");
    }
    mark(c, 6);
    hip_check(c, hipMemcpyAsync(c->host + 8, F.err, sizeof(int32_t), hipMemcpyDeviceToHost,
                                c->stream),
              "read flags");
    sync(c, "fill pass");
    if (reinterpret_cast<const int32_t *>(c->host + 8)[0] & kErrInternal) {
        set_err(c, "internal error: inconsistent staged ranges");
        throw Fail{SLINE_EDEVICE};
    }
    if (c->profile) c->stats.ms_fill = span_ms(c, 5, 6);
}

// Batch with library-allocated outputs: per-graph pair ranges from the task
// offsets, one allocation per graph, and a fill that writes every pair into
// its graph's arrays with the graph's item base taken off both ids (no
// combined result, no split copy).
void run_fill_direct(sline_ctx *c, int64_t total) {
    auto &P = c->bpend;
    const int32_t G = c->direct.G;
    const bool weights = !c->no_weights;
    hipStream_t st = c->stream;
    CountArgs F = c->fill_args;
    P.off.assign(G + 1, 0);
    if (total > 0) {
        hip_check(c, launch_batch_graph_off(st, F.task_item, F.n_tasks, F.task_off, P.ibase_dev, G,
                                            P.off_dev),
                  "graph pair offsets");
        hip_check(c, hipMemcpyAsync(P.off.data(), P.off_dev, sizeof(int64_t) * (G + 1),
                                    hipMemcpyDeviceToHost, st),
                  "read graph pair offsets");
        sync(c, "graph pair offsets");
        if (P.off[0] != 0 || P.off[G] != total) {
            set_err(c, "internal error: graph pair offsets do not cover the result");
            throw Fail{SLINE_EDEVICE};
        }
    }
    std::vector<int32_t *> tab(3 * (size_t)G, nullptr);
    int32_t **d_tab = nullptr;
    auto release = [&]() {
        for (int32_t g = 0; g < G; ++g) {
            const size_t bytes = sizeof(int32_t) * (size_t)(P.off[g + 1] - P.off[g]);
            dev_free(c, tab[g], bytes);
            dev_free(c, tab[G + g], bytes);
            dev_free(c, tab[2 * G + g], bytes);
        }
        dev_free(c, d_tab, sizeof(int32_t *) * tab.size());
    };
    try {
        for (int32_t g = 0; g < G; ++g) {
            const int64_t need = P.off[g + 1] - P.off[g];
            if (need < 0) {
                set_err(c, "internal error: graph pair offsets out of order");
                throw Fail{SLINE_EDEVICE};
            }
            if (need == 0) continue;
            const size_t bytes = sizeof(int32_t) * (size_t)need;
            tab[g] = (int32_t *)dev_alloc(c, bytes);
            tab[G + g] = (int32_t *)dev_alloc(c, bytes);
            tab[2 * G + g] = weights ? (int32_t *)dev_alloc(c, bytes) : nullptr;
            if (!tab[g] || !tab[G + g] || (weights && !tab[2 * G + g])) {
                set_err(c, "output allocation for graph %s failed", std::to_string(g).c_str());
                throw Fail{SLINE_ENOMEM};
            }
        }
        if (total > 0) {
            d_tab = (int32_t **)dev_alloc(c, sizeof(int32_t *) * tab.size());
            if (!d_tab) {
                set_err(c, "output table allocation failed");
                throw Fail{SLINE_ENOMEM};
            }
            hip_check(c, hipMemcpyAsync(d_tab, tab.data(), sizeof(int32_t *) * tab.size(),
                                        hipMemcpyHostToDevice, st),
                      "upload output table");
            F.out_a = F.out_b = F.out_w = nullptr;
            F.n_graphs = G;
            F.g_ibase = P.ibase_dev;
            F.g_off = P.off_dev;
            F.g_out = d_tab;
            fill_into(c, F);  // waits for the stream: the table upload is done too
            dev_free(c, d_tab, sizeof(int32_t *) * tab.size());
            d_tab = nullptr;
        }
    } catch (...) {
        release();
        throw;
    }
    for (int32_t g = 0; g < G; ++g) {
        sline_edges &o = c->direct.outs[g];
        o.n_pairs = P.off[g + 1] - P.off[g];
        o.a = tab[g];
        o.b = tab[G + g];
        o.w = tab[2 * G + g];
    }
    c->direct.done = true;
}

void run_fill(sline_ctx *c, sline_edges *out, int64_t total) {
    if (c->direct.G > 0) {
        run_fill_direct(c, total);
        out->n_pairs = total;
        return;
    }
    const bool weights = !c->no_weights;
    int32_t *a = out->a, *b = out->b, *w = weights ? out->w : nullptr;
    bool owned = false;
    if (out->capacity == 0 && total > 0) {
        const size_t bytes = sizeof(int32_t) * (size_t)total;
        a = (int32_t *)dev_alloc(c, bytes);
        b = a ? (int32_t *)dev_alloc(c, bytes) : nullptr;
        w = (b && weights) ? (int32_t *)dev_alloc(c, bytes) : nullptr;
        if (!b || (weights && !w)) {
            dev_free(c, a, bytes);
            dev_free(c, b, bytes);
            set_err(c, "output allocation of %s pairs failed", std::to_string(total).c_str());
            throw Fail{SLINE_ENOMEM};
        }
        owned = true;
    }
    if (total > 0) {
        CountArgs F = c->fill_args;
        F.out_a = a;
        F.out_b = b;
        F.out_w = w;
        try {
            fill_into(c, F);
        } catch (...) {
            if (owned) {
                const size_t bytes = sizeof(int32_t) * (size_t)total;
                dev_free(c, a, bytes);
                dev_free(c, b, bytes);
                dev_free(c, w, bytes);
            }
            throw;
        }
    }
    if (out->capacity == 0) {
        out->a = owned ? a : nullptr;
        out->b = owned ? b : nullptr;
        out->w = owned ? w : nullptr;
    }
    out->n_pairs = total;
}

// Per-item thresholds of a batch: every item carries its own s (s_item, on
// the device), between s_min and s_max.  Null for a plain build.
struct ItemS {
    const int32_t *s_item = nullptr;
    const int32_t *item_end = nullptr;  // one past the last item of each item's graph
    int32_t s_min = 1, s_max = 1;
    bool full = false;  // product mode (the SpGEMM companion): every b, b = a included
};

sline_status build_core(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual, uint32_t flags,
                        sline_edges *out, const ItemS &IS);
sline_status relabel_impl(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual,
                          uint32_t flags, sline_edges *out);
sline_status intersect_build(sline_ctx *c, const int32_t *ptrI, const int32_t *memI,
                             const int32_t *ptrS, const int32_t *itmS, const int32_t *start,
                             int32_t N, int32_t s, uint32_t flags, int32_t *cnt, int64_t *off,
                             int64_t *part64, unsigned long long *inters, sline_edges *out,
                             sline_stats &S);

// Flags that only a plain single-graph build understands.
constexpr uint32_t kBuildOnlyFlags = SLINE_RELABEL_DESC | SLINE_RELABEL_ASC | SLINE_NO_PRUNE |
                                     SLINE_NO_VISITED | SLINE_NO_SHORTCUT;

sline_status build_impl(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual, uint32_t flags,
                        sline_edges *out) {
    if (!out) {
        set_err(c, "out is NULL");
        return SLINE_EINVAL;
    }
    if (s < 1 || (dual != 0 && dual != 1) || H.n_edges < 0 || H.n_vertices < 0) {
        set_err(c, "invalid argument (s >= 1, dual in {0,1}, sizes >= 0 required)");
        return SLINE_EINVAL;
    }
    if (out->capacity < 0 ||
        (out->capacity > 0 && (!out->a || !out->b || (!out->w && !(flags & SLINE_NO_WEIGHTS))))) {
        set_err(c, "output buffers: capacity > 0 requires a, b and (without SLINE_NO_WEIGHTS) w");
        return SLINE_EINVAL;
    }
    if (flags & (SLINE_RELABEL_DESC | SLINE_RELABEL_ASC)) {
        c->pending.valid = false;
        release_pool(c);
        return relabel_impl(c, H, s, dual, flags, out);
    }
    if (same_call(c->pending, H, s, dual, flags)) {
        const int64_t total = c->pending.total;
        if (out->capacity > 0 && out->capacity < total) {
            out->n_pairs = total;
            set_err(c, "capacity too small");
            return SLINE_ECAPACITY;
        }
        c->pending.valid = false;
        run_fill(c, out, total);
        release_pool(c);
        return SLINE_OK;
    }
    c->pending.valid = false;
    release_pool(c);
    ItemS IS;
    IS.s_min = IS.s_max = s;
    return build_core(c, H, s, dual, flags, out, IS);
}

// sline_build into caller buffers with every device buffer of the build
// carved from this device's scratch array: no allocation, no free.  The
// context's own workspace and any staging pool kept for a capacity retry are
// set aside and put back afterwards untouched.
sline_status noalloc_impl(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual,
                          uint32_t flags, sline_edges *out) {
    if (!out) {
        set_err(c, "out is NULL");
        return SLINE_EINVAL;
    }
    if (s < 1 || (dual != 0 && dual != 1) || H.n_edges < 0 || H.n_vertices < 0) {
        set_err(c, "invalid argument (s >= 1, dual in {0,1}, sizes >= 0 required)");
        return SLINE_EINVAL;
    }
    if (out->capacity <= 0 || !out->a || !out->b || (!out->w && !(flags & SLINE_NO_WEIGHTS))) {
        set_err(c, "sline_build_noalloc writes into caller buffers only: capacity > 0 and a, b "
                   "and (without SLINE_NO_WEIGHTS) w are required");
        return SLINE_EINVAL;
    }
    if (flags & kBuildOnlyFlags) {
        set_err(c, "sline_build_noalloc takes neither relabeling nor the ablation flags");
        return SLINE_EINVAL;
    }
    void *base = scratch_address(c->device);
    if (!base) {
        set_err(c, "the device address of the scratch array could not be taken");
        return SLINE_EDEVICE;
    }
    // a pending capacity retry of sline_build refers to buffers this call reuses
    c->pending.valid = false;
    struct Saved {
        sline_ctx *c;
        void *ws, *ws2, *pool;
        size_t ws_bytes, ws2_bytes, pool_bytes;
        ~Saved() {
            c->fixed = sline_ctx::Fixed{};
            c->pool_fixed = false;
            c->ws = ws;
            c->ws_bytes = ws_bytes;
            c->ws2 = ws2;
            c->ws2_bytes = ws2_bytes;
            c->pool = pool;
            c->pool_bytes = pool_bytes;
        }
    } saved{c, c->ws, c->ws2, c->pool, c->ws_bytes, c->ws2_bytes, c->pool_bytes};
    c->pool = nullptr;
    c->pool_bytes = 0;
    c->pool_fixed = false;
    c->fixed.base = static_cast<char *>(base);
    c->fixed.size = SLINE_NOALLOC_SCRATCH_BYTES;
    c->fixed.used = 0;
    ItemS IS;
    IS.s_min = IS.s_max = s;
    const sline_status r = build_core(c, H, s, dual, flags, out, IS);
    // the counted work lives in the scratch array, which the next call reuses
    c->pending.valid = false;
    release_pool(c);
    return r;
}

sline_status build_core(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual, uint32_t flags,
                        sline_edges *out, const ItemS &IS) {
    c->profile = (flags & SLINE_PROFILE) != 0;
    const int64_t m = H.n_edges, n = H.n_vertices;
    if (m > 0 && !H.row_ptr) {
        set_err(c, "row_ptr is NULL");
        return SLINE_EINVAL;
    }
    hipStream_t st = c->stream;
    sline_stats S{};
    S.n_items = dual ? n : m;
    int64_t nnz = 0;
    // 1. row_ptr check and nnz
    {
        ensure_ws(c, 4096);
        int32_t *err = reinterpret_cast<int32_t *>(c->ws);
        hip_check(c, launch_fill_i32(st, err, 4, 0), "zero flags");
        if (m > 0) {
            hip_check(c, launch_check_rowptr(st, H.row_ptr, (int32_t)m, err), "row_ptr check");
            hip_check(c, hipMemcpyAsync(c->host, H.row_ptr + m, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                      "read nnz");
        } else {
            reinterpret_cast<int32_t *>(c->host)[0] = 0;
        }
        hip_check(c, hipMemcpyAsync(reinterpret_cast<int32_t *>(c->host) + 1, err, sizeof(int32_t),
                                    hipMemcpyDeviceToHost, st),
                  "read flags");
        sync(c, "row_ptr check");
        const int32_t *hp = reinterpret_cast<const int32_t *>(c->host);
        nnz = hp[0];
        if (hp[1] != 0 || nnz < 0) {
            set_err(c, "row_ptr must start at 0 and never decrease");
            return SLINE_EINVAL;
        }
        if (nnz > 0 && !H.col_idx) {
            set_err(c, "col_idx is NULL with nnz > 0");
            return SLINE_EINVAL;
        }
        if (nnz > 0 && n == 0) {
            set_err(c, "members present but n_vertices = 0");
            return SLINE_EINVAL;
        }
    }
    S.nnz = nnz;
    const int64_t N = dual ? n : m;
    const int64_t M = dual ? m : n;
    if (nnz == 0) {
        // no item has a member, so no two items overlap
        c->stats = S;
        out->n_pairs = 0;
        if (out->capacity == 0) out->a = out->b = out->w = nullptr;
        return SLINE_OK;
    }
    const bool noprune = (flags & SLINE_NO_PRUNE) != 0;
    const bool filt = IS.s_max > 1 && !noprune;
    Arena sizing;
    plan_layout(sizing, m, n, nnz, N, M, filt);
    ensure_ws(c, sizing.off + 4096);
    Arena A;
    A.base = reinterpret_cast<char *>(c->ws);
    const Layout L = plan_layout(A, m, n, nnz, N, M, filt);

    hip_check(c, launch_fill_i32(st, L.err, 4, 0), "zero flags");
    hip_check(c, launch_fill_i32(st, L.tcounts, 4, 0), "zero task counts");
    hip_check(c, launch_fill_i64(st, L.totals, 4, 0), "zero totals");
    hip_check(c, launch_fill_i64(st, L.passes, 4, 0), "zero passes");

    mark(c, 0);
    // 2. row ids and member checks (range checks always: they guard every later index)
    hip_check(c, launch_rows(st, H.row_ptr, H.col_idx, (int32_t)m, (int32_t)n, nnz,
                             (flags & SLINE_SKIP_VALIDATE) ? 0 : 1, L.rowid, L.err),
              "row check");
    // 3. transpose (bad members are skipped by every kernel and reported below)
    transpose(c, L, H.col_idx, (int32_t)n, nnz);
    hip_check(c, hipMemcpyAsync(c->host, L.err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read flags");
    sync(c, "member check");
    if (reinterpret_cast<const int32_t *>(c->host)[0] & (kErrColRange | kErrColOrder)) {
        set_err(c, "col_idx: members must lie in [0, n_vertices) and increase strictly within a row");
        return SLINE_EINVAL;
    }
    mark(c, 1);
    // 4. roles
    const int32_t *ptrI = dual ? L.ptrT : H.row_ptr;
    const int32_t *memI = dual ? L.colT : H.col_idx;
    const int32_t *ptrM = dual ? H.row_ptr : L.ptrT;
    const int32_t *itmM = dual ? H.col_idx : L.colT;
    // back-pointer maps: item incidence -> member-list position, and back
    const int32_t *map = dual ? L.kT : L.posT;
    const int32_t *inv = dual ? L.posT : L.kT;
    // 5. s filter
    const int32_t *ptrS = ptrM, *itmS = itmM;
    if (filt) {
        // the task counts are written later: until then their array holds
        // the filter's per-item keep flags
        hip_check(c, launch_filter(st, ptrM, itmM, (int32_t)M, nnz, ptrI, (int32_t)N, s, IS.s_item,
                                   L.ntask, L.pos, L.part32, L.ptrS, L.itmS, inv, L.start),
                  "filter");
        ptrS = L.ptrS;
        itmS = L.itmS;
    }
    // 6. wedge counts, tasks
    const Tuning tu = build_tuning(c->tune, N);
    if (!filt && !IS.full)
        hip_check(c, launch_start_from_map(st, nnz, map, L.start), "back-pointers");
    // degree-based pruning (Sec. IV-C) unless switched off: items smaller
    // than s get no cost and are never walked from
    hip_check(c, launch_cost(st, ptrI, memI, (int32_t)N, noprune ? 1 : s,
                             noprune ? nullptr : IS.s_item, ptrS, itmS, L.cost, L.start,
                             L.totals, IS.full ? 1 : 0, IS.full ? 0 : 1),
              "cost");
    if (flags & SLINE_NO_VISITED) {
        // one set intersection per wedge instead of the counter table
        hip_check(c, launch_fill_i64(st, L.passes, 4, 0), "zero counters");
        int64_t *h = c->host;
        hip_check(c, hipMemcpyAsync(h + 1, L.totals, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st),
                  "read totals");
        sync(c, "wedge totals");
        S.n_kept = h[1];
        S.nnz_kept = h[2];
        S.wedges = h[3];
        if (c->profile) S.ms_transpose = span_ms(c, 0, 1);
        return intersect_build(c, ptrI, memI, ptrS, itmS, L.start, (int32_t)N, s, flags, L.ntask,
                               L.tbase, L.part64, reinterpret_cast<unsigned long long *>(L.passes),
                               out, S);
    }
    if (!(flags & SLINE_NO_SHORTCUT))
        hip_check(c, launch_mark_lookup(st, ptrI, memI, (int32_t)N, s, IS.s_item, IS.s_max, ptrS,
                                        L.start, L.cost, IS.full ? 0 : tu.tiny_max_wedges),
                  "lookup members");
    hip_check(c, launch_task_count(st, L.cost, (int32_t)N, tu, ptrI, IS.item_end, IS.full ? 1 : 0,
                                   L.ntask),
              "task count");
    hip_check(c, launch_scan_i32_to_i64(st, L.ntask, N, L.tbase, L.part64), "task scan");
    int64_t *h = c->host;
    hip_check(c, hipMemcpyAsync(h + 0, L.tbase + N, sizeof(int64_t), hipMemcpyDeviceToHost, st), "read tasks");
    hip_check(c, hipMemcpyAsync(h + 1, L.totals, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st), "read totals");
    sync(c, "task plan");
    const int64_t T = h[0];
    S.n_kept = h[1];
    S.nnz_kept = h[2];
    S.wedges = h[3];
    if (T >= INT32_MAX) {
        set_err(c, "too many counting tasks (%s)", std::to_string(T).c_str());
        throw Fail{SLINE_ENOMEM};
    }
    Arena tsz;
    plan_tasks(tsz, T);
    ensure_ws2(c, tsz.off + 4096);
    Arena TA;
    TA.base = reinterpret_cast<char *>(c->ws2);
    const TaskLayout TL = plan_tasks(TA, T);
    hip_check(c, launch_task_fill(st, L.cost, (int32_t)N, tu, ptrI, IS.item_end, IS.full ? 1 : 0,
                                  L.tbase, TL.item, TL.part, TL.small,
                                  TL.small_item, TL.tiny, TL.tiny_item, TL.big, L.tcounts),
              "task fill");
    mark(c, 2);
    // 7. one counting pass: pairs per task, each range's pairs staged in a pool
    const int64_t want_pool = S.wedges / IS.s_min;  // every pair of L_s accounts for >= s wedges
    // the product route counts and fills in two passes (symbolic, then
    // numeric), as SpGEMM does: its product is too large to stage as well
    c->no_weights = (flags & SLINE_NO_WEIGHTS) != 0;
    const int64_t pool_cap =
        (want_pool > 0 && !IS.full) ? acquire_pool(c, want_pool, c->no_weights ? 4 : 8) : 0;
    hip_check(c, launch_fill_i32(st, TL.need, T, 0), "zero flags");
    // unused records of a reserved log chunk must read as empty
    hip_check(c, launch_fill_i32(st, reinterpret_cast<int32_t *>(TL.log),
                                 (int64_t)TL.log_cap * (int64_t)(sizeof(StageRec) / 4), 0),
              "zero log");
    hip_check(c, launch_fill_i32(st, TL.ctrs, 4, 0), "zero counters");
    hip_check(c, launch_fill_i64(st, reinterpret_cast<int64_t *>(TL.pool_head), 1, 0), "zero pool head");
    CountArgs C{};
    C.mode = pool_cap > 0 ? kModeStage : kModeCount;
    C.ptrI = ptrI;
    C.memI = memI;
    C.ptrS = ptrS;
    C.itmS = itmS;
    C.N = (int32_t)N;
    C.s = s;
    C.s_item = IS.s_item;
    C.item_end = IS.item_end;
    C.full = IS.full ? 1 : 0;
    C.cost = L.cost;
    C.start = L.start;
    C.task_item = TL.item;
    C.task_part = TL.part;
    C.n_tasks = (int32_t)T;
    C.small_tasks = TL.small;
    C.small_items = TL.small_item;
    C.tiny_tasks = TL.tiny;
    C.tiny_items = TL.tiny_item;
    C.big_tasks = TL.big;
    C.task_counts = L.tcounts;
    C.queue = L.queue;
    C.task_cnt = TL.cnt;
    C.task_off = nullptr;
    C.pool_b = reinterpret_cast<int32_t *>(c->pool);
    C.pool_w = (c->pool && !c->no_weights) ? reinterpret_cast<int32_t *>(c->pool) + pool_cap : nullptr;
    C.pool_cap = pool_cap;
    C.pool_head = TL.pool_head;
    C.log = TL.log;
    C.log_cap = TL.log_cap;
    {
        // chunks small enough that every resident workgroup gets several
        const int64_t groups = (int64_t)c->n_cu * (tu.small_grid_per_cu + tu.task_grid_per_cu);
        C.pool_chunk = std::max<int64_t>(256, std::min<int64_t>(1 << 16, pool_cap / (8 * groups)));
        C.log_chunk = (int32_t)std::max<int64_t>(
            1, std::min<int64_t>(256, (int64_t)TL.log_cap / (8 * groups)));
    }
    C.log_head = TL.ctrs;
    C.need = TL.need;
    C.need_count = TL.ctrs + 1;
    C.passes = L.passes;
    C.err = L.err;
    C.tune = tu;
    C.n_cu = c->n_cu;
    hip_check(c, launch_count(st, C, c->profile ? c->ev[7] : nullptr), "count pass");
    mark(c, 3);
    hip_check(c, launch_scan_i32_to_i64(st, TL.cnt, T, TL.off, TL.part64), "pair scan");
    mark(c, 4);
    hip_check(c, hipMemcpyAsync(h + 0, TL.off + T, sizeof(int64_t), hipMemcpyDeviceToHost, st), "read total");
    hip_check(c, hipMemcpyAsync(h + 4, L.passes, sizeof(int64_t), hipMemcpyDeviceToHost, st), "read passes");
    hip_check(c, hipMemcpyAsync(h + 9, L.passes + 1, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st),
              "read task kernel work");
    hip_check(c, hipMemcpyAsync(h + 12, L.tcounts, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st),
              "read task counts");
    hip_check(c, hipMemcpyAsync(h + 6, L.err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read flags");
    hip_check(c, hipMemcpyAsync(h + 7, TL.ctrs, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st), "read stage counters");
    sync(c, "count pass");
    const int64_t total = h[0];
    const int32_t *hb = reinterpret_cast<const int32_t *>(h + 12);
    const int32_t *hc = reinterpret_cast<const int32_t *>(h + 7);
    S.passes = h[4];
    S.heavy_nnz = h[9];
    S.heavy_wedges = h[10];
    S.heavy_pairs = h[11];
    S.n_small = hb[0] + hb[2];  // one-wave and one-lane items
    S.n_heavy = hb[1];
    S.n_pairs = total;
    if (c->profile) {
        S.ms_transpose = span_ms(c, 0, 1);
        S.ms_prepare = span_ms(c, 1, 2);
        S.ms_count = span_ms(c, 2, 3);
        S.ms_tasks = span_ms(c, 7, 3);
        S.ms_scan = span_ms(c, 3, 4);
    }
    if (reinterpret_cast<const int32_t *>(h + 6)[0] & kErrInternal) {
        set_err(c, "internal error: counting table overflow");
        return SLINE_EDEVICE;
    }
    c->fill_records = C.mode == kModeStage ? std::min(hc[0], TL.log_cap) : 0;
    c->fill_need = C.mode == kModeStage ? hc[1] : -1;
    c->stats = S;
    C.task_off = TL.off;
    C.passes = nullptr;
    c->fill_args = C;
    c->fill_total = total;
    if (out->capacity > 0 && out->capacity < total) {
        c->pending.valid = true;
        c->pending.H = H;
        c->pending.s = s;
        c->pending.dual = dual;
        c->pending.flags = flags;
        c->pending.total = total;
        out->n_pairs = total;
        set_err(c, "capacity too small");
        return SLINE_ECAPACITY;
    }
    // 8. fill
    run_fill(c, out, total);
    release_pool(c);
    return SLINE_OK;
}

}  // namespace

// ---------------------------------------------------------------- batches

namespace {

void drop_batch_pending(sline_ctx *c) {
    auto &P = c->bpend;
    if (P.comb.a) {
        (void)hipStreamSynchronize(c->stream);
        const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(P.comb.n_pairs, 1);
        dev_free(c, P.comb.a, bytes);
        dev_free(c, P.comb.b, bytes);
        dev_free(c, P.comb.w, bytes);
    }
    if (P.bws) dev_free(c, P.bws, P.bws_bytes);
    P = sline_ctx::BatchPending{};
}

bool same_batch(const sline_ctx::BatchPending &P, int32_t G, const sline_csr *Hs, const int32_t *s,
                const int32_t *dual, uint32_t flags) {
    if (!P.valid || (int32_t)P.H.size() != G || P.flags != flags) return false;
    for (int32_t g = 0; g < G; ++g) {
        const sline_csr &a = P.H[g], &b = Hs[g];
        if (a.row_ptr != b.row_ptr || a.col_idx != b.col_idx || a.n_edges != b.n_edges ||
            a.n_vertices != b.n_vertices || P.s[g] != s[g] || P.dual[g] != dual[g])
            return false;
    }
    return true;
}

// Hand each graph its slice of the combined result (ids shifted back), into
// caller buffers or freshly allocated ones; checks capacities first.
sline_status batch_split(sline_ctx *c, int32_t G, sline_edges *outs) {
    auto &P = c->bpend;
    hipStream_t st = c->stream;
    for (int32_t g = 0; g < G; ++g) {
        const int64_t need = P.off[g + 1] - P.off[g];
        if (outs[g].capacity > 0 && outs[g].capacity < need) {
            for (int32_t h = 0; h < G; ++h) outs[h].n_pairs = P.off[h + 1] - P.off[h];
            set_err(c, "capacity too small for at least one graph");
            return SLINE_ECAPACITY;
        }
    }
    if (G == 1 && outs[0].capacity == 0) {
        // one graph: its items start at id 0, so the combined arrays are its result
        outs[0].n_pairs = P.comb.n_pairs;
        outs[0].a = P.comb.a;
        outs[0].b = P.comb.b;
        outs[0].w = P.comb.w;
        P.comb = sline_edges{};
        return SLINE_OK;
    }
    std::vector<int32_t *> pa(G), pb(G), pw(G);
    std::vector<char> owned(G, 0);
    try {
        for (int32_t g = 0; g < G; ++g) {
            const int64_t need = P.off[g + 1] - P.off[g];
            if (outs[g].capacity > 0) {
                pa[g] = outs[g].a;
                pb[g] = outs[g].b;
                pw[g] = outs[g].w;
            } else if (need > 0) {
                const size_t bytes = sizeof(int32_t) * (size_t)need;
                pa[g] = (int32_t *)dev_alloc(c, bytes);
                pb[g] = (int32_t *)dev_alloc(c, bytes);
                pw[g] = (P.flags & SLINE_NO_WEIGHTS) ? nullptr : (int32_t *)dev_alloc(c, bytes);
                owned[g] = 1;
                if (!pa[g] || !pb[g] || (!pw[g] && !(P.flags & SLINE_NO_WEIGHTS))) {
                    set_err(c, "output allocation failed");
                    throw Fail{SLINE_ENOMEM};
                }
            }
        }
        if (P.comb.n_pairs > 0) {
            int32_t **ptrs = (int32_t **)dev_alloc(c, sizeof(int32_t *) * 3 * (size_t)G);
            if (!ptrs) {
                set_err(c, "output table allocation failed");
                throw Fail{SLINE_ENOMEM};
            }
            std::vector<int32_t *> h(3 * (size_t)G);
            for (int32_t g = 0; g < G; ++g) {
                h[g] = pa[g];
                h[G + g] = pb[g];
                h[2 * G + g] = pw[g];
            }
            hipError_t e = hipMemcpyAsync(ptrs, h.data(), sizeof(int32_t *) * h.size(),
                                          hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = launch_batch_split(st, P.ibase_dev, P.off_dev, G, P.comb.a, P.comb.b, P.comb.w,
                                       P.comb.n_pairs, ptrs, ptrs + G, ptrs + 2 * G);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            dev_free(c, ptrs, sizeof(int32_t *) * 3 * (size_t)G);
            hip_check(c, e, "batch split");
        }
    } catch (...) {
        for (int32_t g = 0; g < G; ++g) {
            if (!owned[g]) continue;
            const size_t bytes = sizeof(int32_t) * (size_t)(P.off[g + 1] - P.off[g]);
            dev_free(c, pa[g], bytes);
            dev_free(c, pb[g], bytes);
            dev_free(c, pw[g], bytes);
        }
        throw;
    }
    for (int32_t g = 0; g < G; ++g) {
        outs[g].n_pairs = P.off[g + 1] - P.off[g];
        if (outs[g].capacity == 0) {
            outs[g].a = pa[g];
            outs[g].b = pb[g];
            outs[g].w = pw[g];
        }
    }
    return SLINE_OK;
}

// Combined sizes of a batch and the bases of every graph in them (its first
// combined item and member; for dual graphs, its first row and entry in XD,
// the row concatenation of the dual graphs, and its first row of XD^T).
struct BatchBases {
    std::vector<int64_t> ibase, dbase;  // ibase: G + 1 entries; dbase: GD + 1
    std::vector<int32_t> dual_ids;      // the dual graphs, in order
    int64_t NI = 0, MT = 0, ZT = 0, E = 0, ZD = 0, VD = 0;
    int32_t GD() const { return (int32_t)dual_ids.size(); }
};

// Sets every descriptor's nnz and bases from the graphs' nnz.  SLINE_EINVAL
// (error set) for a bad nnz, a missing col_idx, or combined counts of 2^31 or
// more.
sline_status batch_bases(sline_ctx *c, std::vector<BatchGraph> &gr, const std::vector<int64_t> &nnz,
                         BatchBases &B) {
    const int32_t G = (int32_t)gr.size();
    B = BatchBases{};
    B.ibase.assign(G + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
        BatchGraph &d = gr[g];
        if (nnz[g] < 0 || (nnz[g] > 0 && (!d.col || d.n == 0))) {
            set_err(c, "graph %s: bad nnz or missing col_idx", std::to_string(g).c_str());
            return SLINE_EINVAL;
        }
        d.nnz = nnz[g];
        d.ibase = B.NI;
        d.mbase = B.MT;
        B.ibase[g] = B.NI;
        B.NI += d.dual ? d.n : d.m;
        B.MT += d.dual ? d.m : d.n;
        B.ZT += nnz[g];
        if (d.dual) {
            d.dbase = B.E;
            d.dzbase = B.ZD;
            d.vdbase = B.VD;
            B.dual_ids.push_back(g);
            B.dbase.push_back(B.E);
            B.E += d.m;
            B.ZD += nnz[g];
            B.VD += d.n;
        }
    }
    B.ibase[G] = B.NI;
    B.dbase.push_back(B.E);
    if (B.NI >= INT32_MAX || B.MT >= INT32_MAX || B.ZT >= INT32_MAX) {
        set_err(c, "batch too large: combined items, members and incidences must stay below 2^31");
        return SLINE_EINVAL;
    }
    return SLINE_OK;
}

// Arrays of the combine stage: XD and its transpose, then the combined item
// CSR with every item's s and graph end.
struct Combine {
    Layout X{};
    int32_t *len = nullptr, *ptrC = nullptr, *memC = nullptr, *s_item = nullptr, *iend = nullptr;
};

Combine plan_combine(Arena &A, const BatchBases &B) {
    Combine K;
    K.X.rowid = A.take<int32_t>(B.ZD);
    K.X.colT = A.take<int32_t>(B.ZD);
    K.X.ptrT = A.take<int32_t>(B.VD + 1);
    K.X.rsK0 = A.take<int32_t>(B.ZD);
    K.X.rsK1 = A.take<int32_t>(B.ZD);
    K.X.rsV0 = A.take<int32_t>(B.ZD);
    K.X.rsV1 = A.take<int32_t>(B.ZD);
    K.X.rsHist = A.take<int32_t>(transpose_hist(B.ZD));
    K.X.part32 = A.take<int32_t>(scan_partials(std::max<int64_t>({B.VD, B.NI, B.ZD}) + 1));
    K.len = A.take<int32_t>(B.NI);
    K.ptrC = A.take<int32_t>(B.NI + 1);
    K.memC = A.take<int32_t>(B.ZT);
    K.s_item = A.take<int32_t>(B.NI);
    K.iend = A.take<int32_t>(B.NI);
    K.X.xcol = A.take<int32_t>(B.ZD);
    return K;
}

// Device copies of the descriptors and bases the combine stage reads.
struct BatchDev {
    const BatchGraph *gr;
    const int64_t *ibase, *dbase;
    const int32_t *dual_ids;
    int32_t *zb;   // G + 1 entries
    int32_t *err;  // CSR rule violations (kErr* bits)
};

// Enqueue the combine stage on `st`: the dual graphs' rows concatenated and
// transposed, then every combined item's list, s and graph end, with the
// checks of every caller CSR (bits in D.err).
void enqueue_combine(sline_ctx *c, hipStream_t st, int32_t G, const BatchBases &B,
                     const BatchDev &D, const Combine &K) {
    const Layout &X = K.X;
    hip_check(c, launch_fill_i32(st, X.xcol, B.ZD, 0), "zero dual columns");
    hip_check(c, launch_fill_i32(st, X.rowid, B.ZD, 0), "zero dual rows");
    if (B.GD() > 0 && B.E > 0) {
        hip_check(c, launch_batch_concat(st, D.gr, D.dual_ids, D.dbase, B.GD(), B.E, X.xcol, X.rowid,
                                         D.err),
                  "dual rows");
        if (B.ZD > 0) {
            int32_t *const rk[2] = {X.rsK0, X.rsK1};
            int32_t *const rv[2] = {X.rsV0, X.rsV1};
            hip_check(c, launch_transpose(st, X.xcol, B.ZD, (int32_t)B.VD, X.rowid, rk, rv, X.rsHist,
                                          X.part32, X.ptrT, X.colT, nullptr, nullptr),
                      "dual transpose");
        } else {
            hip_check(c, launch_fill_i32(st, X.ptrT, B.VD + 1, 0), "empty transpose");
        }
    } else if (B.VD > 0) {
        hip_check(c, launch_fill_i32(st, X.ptrT, B.VD + 1, 0), "empty transpose");
    }
    hip_check(c, launch_batch_len(st, D.gr, D.ibase, G, B.NI, X.ptrT, K.len, K.s_item, K.iend,
                                  D.err),
              "item lengths");
    hip_check(c, launch_scan_i32(st, K.len, B.NI, K.ptrC, X.part32), "item scan");
    hip_check(c, launch_batch_rows(st, D.gr, D.ibase, G, B.ZT, X.ptrT, X.colT, K.ptrC, D.zb,
                                   K.memC, D.err),
              "item rows");
}

sline_status batch_impl(sline_ctx *c, int32_t G, const sline_csr *Hs, const int32_t *s,
                        const int32_t *dual, uint32_t flags, sline_edges *outs) {
    if (flags & kBuildOnlyFlags) {
        set_err(c, "relabeling and the ablation flags apply to sline_build only");
        return SLINE_EINVAL;
    }
    if (G < 0 || (G > 0 && (!Hs || !s || !dual || !outs))) {
        set_err(c, "invalid batch arguments");
        return SLINE_EINVAL;
    }
    for (int32_t g = 0; g < G; ++g) {
        const sline_csr &H = Hs[g];
        if (s[g] < 1 || (dual[g] != 0 && dual[g] != 1) || H.n_edges < 0 || H.n_vertices < 0 ||
            (H.n_edges > 0 && !H.row_ptr) || outs[g].capacity < 0 ||
            (outs[g].capacity > 0 &&
             (!outs[g].a || !outs[g].b || (!outs[g].w && !(flags & SLINE_NO_WEIGHTS))))) {
            set_err(c, "invalid arguments for graph %s", std::to_string(g).c_str());
            return SLINE_EINVAL;
        }
    }
    if (same_batch(c->bpend, G, Hs, s, dual, flags)) {
        const sline_status r = batch_split(c, G, outs);
        if (r == SLINE_OK) drop_batch_pending(c);
        return r;
    }
    drop_batch_pending(c);
    c->pending.valid = false;
    if (G == 0) return SLINE_OK;
    hipStream_t st = c->stream;
    auto &P = c->bpend;
    // 1. per-graph nnz and row_ptr[0] checks
    std::vector<BatchGraph> gr(G);
    int32_t s_min = INT32_MAX, s_max = 1;
    for (int32_t g = 0; g < G; ++g) {
        BatchGraph &d = gr[g];
        d = BatchGraph{};
        d.rp = Hs[g].row_ptr;
        d.col = Hs[g].col_idx;
        d.m = Hs[g].n_edges;
        d.n = Hs[g].n_vertices;
        d.dual = dual[g];
        d.s = s[g];
        s_min = std::min(s_min, s[g]);
        s_max = std::max(s_max, s[g]);
    }
    // small workspace: descriptors, nnz, flags, item bases, pair offsets, dual lists
    const size_t small = sizeof(BatchGraph) * G + 8 * (size_t)(5 * G + 16) + 4096;
    P.bws_bytes = small;
    P.bws = dev_alloc(c, small);
    if (!P.bws) {
        set_err(c, "batch workspace allocation failed");
        throw Fail{SLINE_ENOMEM};
    }
    Arena W;
    W.base = reinterpret_cast<char *>(P.bws);
    BatchGraph *d_gr = W.take<BatchGraph>(G);
    int64_t *d_nnz = W.take<int64_t>(G);
    int32_t *d_err = W.take<int32_t>(4);
    P.ibase_dev = W.take<int64_t>(G + 1);
    P.off_dev = W.take<int64_t>(G + 1);
    int64_t *d_dbase = W.take<int64_t>(G + 1);
    int32_t *d_dual_ids = W.take<int32_t>(G);
    int32_t *d_zb = W.take<int32_t>(G + 1);
    hip_check(c, launch_fill_i32(st, d_err, 4, 0), "zero flags");
    hip_check(c, hipMemcpyAsync(d_gr, gr.data(), sizeof(BatchGraph) * G, hipMemcpyHostToDevice, st),
              "upload graphs");
    hip_check(c, launch_batch_nnz(st, d_gr, G, d_nnz, d_err), "batch nnz");
    std::vector<int64_t> nnz(G);
    int32_t herr = 0;
    hip_check(c, hipMemcpyAsync(nnz.data(), d_nnz, sizeof(int64_t) * G, hipMemcpyDeviceToHost, st),
              "read nnz");
    hip_check(c, hipMemcpyAsync(&herr, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read flags");
    sync(c, "batch nnz");
    if (herr) {
        set_err(c, "row_ptr must start at 0 in every graph");
        drop_batch_pending(c);
        return SLINE_EINVAL;
    }
    // 2. bases on the host
    BatchBases B;
    if (batch_bases(c, gr, nnz, B) != SLINE_OK) {
        drop_batch_pending(c);
        return SLINE_EINVAL;
    }
    const int64_t NI = B.NI, MT = B.MT;
    const int32_t GD = B.GD();
    hip_check(c, hipMemcpyAsync(d_gr, gr.data(), sizeof(BatchGraph) * G, hipMemcpyHostToDevice, st),
              "upload graphs");
    hip_check(c, hipMemcpyAsync(P.ibase_dev, B.ibase.data(), sizeof(int64_t) * (G + 1),
                                hipMemcpyHostToDevice, st),
              "upload item bases");
    if (GD > 0) {
        hip_check(c, hipMemcpyAsync(d_dbase, B.dbase.data(), sizeof(int64_t) * (GD + 1),
                                    hipMemcpyHostToDevice, st),
                  "upload dual bases");
        hip_check(c, hipMemcpyAsync(d_dual_ids, B.dual_ids.data(), sizeof(int32_t) * GD,
                                    hipMemcpyHostToDevice, st),
                  "upload dual ids");
    }
    // 3. XD and its transpose; 4. combined item CSR
    Arena sz;
    (void)plan_combine(sz, B);
    void *big = dev_alloc(c, sz.off + 4096);
    if (!big) {
        set_err(c, "batch arrays allocation failed");
        drop_batch_pending(c);
        throw Fail{SLINE_ENOMEM};
    }
    const size_t big_bytes = sz.off + 4096;
    sline_edges comb{};
    try {
        Arena A;
        A.base = reinterpret_cast<char *>(big);
        const Combine K = plan_combine(A, B);
        enqueue_combine(c, st, G, B, BatchDev{d_gr, P.ibase_dev, d_dbase, d_dual_ids, d_zb, d_err}, K);
        hip_check(c, hipMemcpyAsync(&herr, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read flags");
        sync(c, "batch items");
        if (herr) {
            set_err(c, "a graph breaks the CSR rules (row_ptr order, member range or order)");
            dev_free(c, big, big_bytes);
            drop_batch_pending(c);
            return SLINE_EINVAL;
        }
        // 5. one pass of the pipeline over the combined items, each with its own s
        sline_csr CH{};
        CH.row_ptr = K.ptrC;
        CH.col_idx = K.memC;
        CH.n_edges = (int32_t)NI;
        CH.n_vertices = (int32_t)std::max<int64_t>(MT, 1);
        ItemS IS;
        IS.s_item = K.s_item;
        IS.item_end = K.iend;
        IS.s_min = s_min;
        IS.s_max = s_max;
        // library-allocated outputs of several graphs: the fill writes them
        // directly (one graph takes the combined arrays as they are)
        bool direct = G > 1;
        for (int32_t g = 0; g < G; ++g) direct = direct && outs[g].capacity == 0;
        struct DirectScope {
            sline_ctx *c;
            ~DirectScope() { c->direct = sline_ctx::Direct{}; }
        } scope{c};
        if (direct) {
            for (int32_t g = 0; g < G; ++g) outs[g] = sline_edges{};
            c->direct.G = G;
            c->direct.outs = outs;
        }
        // the combined lists' row check verifies the member order of every
        // primal graph (SLINE_SKIP_VALIDATE, if given, skips it)
        const sline_status r = build_core(c, CH, s_min, 0, flags, &comb, IS);
        if (r == SLINE_OK && c->direct.done) {
            release_pool(c);
            dev_free(c, big, big_bytes);
            drop_batch_pending(c);
            return SLINE_OK;
        }
        if (r != SLINE_OK) {
            dev_free(c, big, big_bytes);
            drop_batch_pending(c);
            return r;
        }
        release_pool(c);
    } catch (...) {
        dev_free(c, big, big_bytes);
        drop_batch_pending(c);
        throw;
    }
    dev_free(c, big, big_bytes);
    // 6. per-graph slices
    P.comb = comb;
    P.off.assign(G + 1, 0);
    if (comb.n_pairs > 0) {
        hip_check(c, launch_batch_bounds(st, P.ibase_dev, G, comb.a, comb.n_pairs, P.off_dev),
                  "graph bounds");
        hip_check(c, hipMemcpyAsync(P.off.data(), P.off_dev, sizeof(int64_t) * (G + 1),
                                    hipMemcpyDeviceToHost, st),
                  "read graph bounds");
        sync(c, "graph bounds");
    }
    P.H.assign(Hs, Hs + G);
    P.s.assign(s, s + G);
    P.dual.assign(dual, dual + G);
    P.flags = flags;
    P.valid = true;
    const sline_status r = batch_split(c, G, outs);
    if (r == SLINE_OK) drop_batch_pending(c);
    return r;
}

// ------------------------------------------------------------ batch plans
//
// A batch whose every buffer is sized once, so that the whole pipeline --
// shape checks, combine stage, transpose, s filter, costs, tasks, one
// counting pass with staging, pair scan, staged copy, recount of tasks that
// found no room, per-graph offsets -- is captured as one HIP graph.  Sizes
// that depend on the data (tasks, pairs) are the ones counted when the plan
// was made; guard kernels compare each run's counts with them and, when a
// count is larger, set a bit that makes every later kernel of the run return
// at once, so that no kernel writes past its buffer.

}  // namespace

struct sline_batch_plan {
    sline_ctx *c = nullptr;
    int32_t G = 0;
    uint32_t flags = 0;
    bool weights = true;
    std::vector<BatchGraph> gr;        // descriptors as last uploaded
    bool gr_stale = false;             // an upload of gr may not have completed
    std::vector<int32_t> s_plan;       // each graph's planned s
    BatchBases B;
    int32_t s_min = 1;
    std::vector<std::pair<void *, size_t>> mem;  // device allocations
    // device views
    BatchGraph *d_gr = nullptr;
    int64_t *d_nnz = nullptr, *ibase = nullptr, *dbase = nullptr, *off = nullptr;
    int32_t *d_err = nullptr, *dual_ids = nullptr, *zb = nullptr;
    Combine K;
    Layout L{};
    TaskLayout TL{};
    CountArgs C{};
    int64_t t_cap = 0, pair_cap = 0, pool_cap = 0;
    int32_t *pool = nullptr, *out_a = nullptr, *out_b = nullptr, *out_w = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t *host = nullptr;  // pinned read-back: off (G + 1 words), then 16 words
};

namespace {

void plan_free(sline_batch_plan *p) {
    if (!p) return;
    sline_ctx *c = p->c;
    if (c) (void)hipStreamSynchronize(c->stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (auto &m : p->mem) dev_free(c, m.first, m.second);
    if (c) (void)hipStreamSynchronize(c->stream);
    if (p->host) (void)hipHostFree(p->host);
    delete p;
}

void *plan_alloc(sline_batch_plan *p, size_t bytes, const char *what) {
    void *q = dev_alloc(p->c, bytes);
    if (!q) {
        set_err(p->c, "batch plan: allocation of %s failed", what);
        throw Fail{SLINE_ENOMEM};
    }
    p->mem.emplace_back(q, bytes);
    return q;
}

BatchDev plan_dev(sline_batch_plan *p) {
    return BatchDev{p->d_gr, p->ibase, p->dbase, p->dual_ids, p->zb, p->d_err};
}

// Shape checks, combine stage, transposes, filter, costs, lookup-only members
// and the task scan; with t_cap >= 0, the guard of the task count.
void plan_enqueue_prep(sline_batch_plan *p, hipStream_t st, int64_t t_cap) {
    sline_ctx *c = p->c;
    const BatchBases &B = p->B;
    hip_check(c, launch_fill_i32(st, p->d_err, 4, 0), "zero flags");
    hip_check(c, launch_plan_check_shape(st, p->d_gr, p->G, p->d_err), "shape check");
    if (B.ZT == 0) {
        hip_check(c, launch_fill_i64(st, p->off, p->G + 1, 0), "zero offsets");
        return;
    }
    enqueue_combine(c, st, p->G, B, plan_dev(p), p->K);
    const Layout &L = p->L;
    const int32_t NI = (int32_t)B.NI, MT = (int32_t)B.MT;
    const int32_t *ptrI = p->K.ptrC, *memI = p->K.memC;
    hip_check(c, launch_fill_i32(st, L.err, 4, 0), "zero flags");
    hip_check(c, launch_fill_i32(st, L.tcounts, 4, 0), "zero task counts");
    hip_check(c, launch_fill_i64(st, L.totals, 4, 0), "zero totals");
    hip_check(c, launch_fill_i64(st, L.passes, 4, 0), "zero passes");
    // row ids, and the member order of every row (a primal graph's combined
    // ids keep its members' order); a violation stops the run's counting
    hip_check(c, launch_rows(st, ptrI, memI, NI, MT, B.ZT, 1, L.rowid, p->d_err), "row ids");
    int32_t *const rk[2] = {L.rsK0, L.rsK1};
    int32_t *const rv[2] = {L.rsV0, L.rsV1};
    hip_check(c, launch_transpose(st, memI, B.ZT, MT, L.rowid, rk, rv, L.rsHist, L.part32, L.ptrT,
                                  L.colT, L.kT, L.posT),
              "transpose");
    // every item carries its graph's s; the filter, the costs and the
    // lookup-only members read them per item, so a run's s need not be the
    // planned one
    hip_check(c, launch_filter(st, L.ptrT, L.colT, MT, B.ZT, ptrI, NI, p->s_min, p->K.s_item,
                               L.ntask, L.pos, L.part32, L.ptrS, L.itmS, L.kT, L.start),
              "filter");
    hip_check(c, launch_cost(st, ptrI, memI, NI, p->s_min, p->K.s_item, L.ptrS, L.itmS, L.cost,
                             L.start, L.totals, 0, 1),
              "cost");
    const Tuning &tu = p->C.tune;
    hip_check(c, launch_mark_lookup(st, ptrI, memI, NI, p->s_min, p->K.s_item, INT32_MAX, L.ptrS,
                                    L.start, L.cost, tu.tiny_max_wedges),
              "lookup members");
    hip_check(c, launch_task_count(st, L.cost, NI, tu, ptrI, p->K.iend, 0, L.ntask), "task count");
    hip_check(c, launch_scan_i32_to_i64(st, L.ntask, NI, L.tbase, L.part64), "task scan");
    if (t_cap >= 0)
        hip_check(c, launch_plan_guard(st, L.tbase + NI, t_cap, kErrPlanTasks, p->d_err), "task guard");
}

// Task lists, the counting pass (staging into the pool) and the pair scan;
// with pair_cap >= 0, the guard of the pair count.
void plan_enqueue_count(sline_batch_plan *p, hipStream_t st, int64_t pair_cap) {
    if (p->B.ZT == 0) return;
    sline_ctx *c = p->c;
    const Layout &L = p->L;
    const TaskLayout &TL = p->TL;
    const CountArgs &C = p->C;
    const int32_t NI = (int32_t)p->B.NI;
    hip_check(c, launch_task_fill(st, L.cost, NI, C.tune, C.ptrI, p->K.iend, 0, L.tbase, TL.item,
                                  TL.part, TL.small, TL.small_item, TL.tiny, TL.tiny_item, TL.big,
                                  L.tcounts, p->d_err),
              "task fill");
    hip_check(c, launch_fill_i32(st, TL.need, p->t_cap, 0), "zero need flags");
    hip_check(c, launch_fill_i32(st, reinterpret_cast<int32_t *>(TL.log),
                                 (int64_t)TL.log_cap * (int64_t)(sizeof(StageRec) / 4), 0),
              "zero log");
    hip_check(c, launch_fill_i32(st, TL.ctrs, 4, 0), "zero counters");
    hip_check(c, launch_fill_i64(st, reinterpret_cast<int64_t *>(TL.pool_head), 1, 0),
              "zero pool head");
    // tasks beyond this run's count must add no pairs to the scan
    hip_check(c, launch_fill_i32(st, TL.cnt, p->t_cap, 0), "zero pair counts");
    hip_check(c, launch_count(st, C), "count pass");
    hip_check(c, launch_scan_i32_to_i64(st, TL.cnt, p->t_cap, TL.off, TL.part64), "pair scan");
    if (pair_cap >= 0)
        hip_check(c, launch_plan_guard(st, TL.off + p->t_cap, pair_cap, kErrPlanPairs, p->d_err),
                  "pair guard");
}

// Staged ranges to the result arrays (each graph's ids less its item base),
// recount of the tasks that found no room, and the per-graph offsets.
void plan_enqueue_fill(sline_batch_plan *p, hipStream_t st) {
    if (p->B.ZT == 0) return;
    sline_ctx *c = p->c;
    CountArgs F = p->C;
    F.task_off = p->TL.off;
    F.passes = nullptr;
    F.out_a = p->out_a;
    F.out_b = p->out_b;
    F.out_w = p->weights ? p->out_w : nullptr;
    F.n_graphs = p->G;
    F.g_ibase = p->ibase;
    F.g_off = nullptr;
    F.g_out = nullptr;
    if (F.mode == kModeStage) {
        hip_check(c, launch_stage_copy(st, F, -1), "stage copy");
        F.mode = kModeFill;  // only the flagged tasks, and nothing when none is
    } else {
        F.mode = kModeFill;
        F.need = nullptr;
    }
    hip_check(c, launch_count(st, F), "fill pass");
    hip_check(c, launch_batch_graph_off(st, p->TL.item, (int32_t)p->t_cap, p->TL.off, p->ibase,
                                        p->G, p->off, p->L.tbase + p->B.NI),
              "graph pair offsets");
}

// Counting arguments of the plan's pass (mode, pool and chunks set by the caller).
CountArgs plan_count_args(sline_batch_plan *p) {
    const Layout &L = p->L;
    const TaskLayout &TL = p->TL;
    CountArgs C = p->C;  // keeps the tuning
    C.ptrI = p->K.ptrC;
    C.memI = p->K.memC;
    C.ptrS = L.ptrS;
    C.itmS = L.itmS;
    C.N = (int32_t)p->B.NI;
    C.s = p->s_min;
    C.s_item = p->K.s_item;
    C.item_end = p->K.iend;
    C.full = 0;
    C.cost = L.cost;
    C.start = L.start;
    C.task_item = TL.item;
    C.task_part = TL.part;
    C.n_tasks = (int32_t)p->t_cap;
    C.small_tasks = TL.small;
    C.small_items = TL.small_item;
    C.tiny_tasks = TL.tiny;
    C.tiny_items = TL.tiny_item;
    C.big_tasks = TL.big;
    C.task_counts = L.tcounts;
    C.queue = L.queue;
    C.task_cnt = TL.cnt;
    C.task_off = nullptr;
    C.pool_b = p->pool;
    C.pool_w = (p->pool && p->weights) ? p->pool + p->pool_cap : nullptr;
    C.pool_cap = p->pool_cap;
    C.pool_head = TL.pool_head;
    C.log = TL.log;
    C.log_cap = TL.log_cap;
    C.log_head = TL.ctrs;
    C.need = TL.need;
    C.need_count = TL.ctrs + 1;
    C.passes = L.passes;
    C.err = L.err;
    C.n_cu = p->c->n_cu;
    C.abort = p->d_err;
    C.mode = p->pool_cap > 0 ? kModeStage : kModeCount;
    const int64_t groups =
        (int64_t)C.n_cu * (C.tune.small_grid_per_cu + C.tune.task_grid_per_cu);
    C.pool_chunk = std::max<int64_t>(256, std::min<int64_t>(1 << 16, p->pool_cap / (8 * groups)));
    C.log_chunk =
        (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, (int64_t)TL.log_cap / (8 * groups)));
    return C;
}

// Staging pool of `pairs` pairs (halving on failure); 0 pairs: no pool.
void plan_pool(sline_batch_plan *p, int64_t pairs) {
    const int64_t pair_bytes = p->weights ? 8 : 4;
    int64_t cap = std::min<int64_t>(pairs, p->C.tune.stage_max_bytes / pair_bytes);
    p->pool = nullptr;
    p->pool_cap = 0;
    while (cap >= 256) {
        void *q = dev_alloc(p->c, (size_t)(cap * pair_bytes));
        if (q) {
            p->mem.emplace_back(q, (size_t)(cap * pair_bytes));
            p->pool = reinterpret_cast<int32_t *>(q);
            p->pool_cap = cap;
            return;
        }
        cap /= 2;
    }
}

void plan_drop_last(sline_batch_plan *p, void *q) {
    for (size_t i = 0; i < p->mem.size(); ++i) {
        if (p->mem[i].first == q) {
            (void)hipStreamSynchronize(p->c->stream);
            dev_free(p->c, q, p->mem[i].second);
            p->mem.erase(p->mem.begin() + (long)i);
            return;
        }
    }
}

sline_status plan_csr_error(sline_ctx *c, int32_t e) {
    if (e & kErrPlanShape)
        set_err(c, "batch plan: a graph's row_ptr[0] or row_ptr[m] differs from the planned one");
    else
        set_err(c, "a graph breaks the CSR rules (row_ptr order, member range or order)");
    return SLINE_EINVAL;
}

sline_status plan_create_impl(sline_ctx *c, int32_t G, const sline_csr *Hs, const int32_t *s,
                              const int32_t *dual, uint32_t flags, sline_batch_plan **out) {
    if (!out) {
        set_err(c, "plan is NULL");
        return SLINE_EINVAL;
    }
    *out = nullptr;
    if (flags & ~(uint32_t)SLINE_NO_WEIGHTS) {
        set_err(c, "batch plans take no flag but SLINE_NO_WEIGHTS");
        return SLINE_EINVAL;
    }
    if (G < 0 || (G > 0 && (!Hs || !s || !dual))) {
        set_err(c, "invalid batch arguments");
        return SLINE_EINVAL;
    }
    for (int32_t g = 0; g < G; ++g) {
        const sline_csr &H = Hs[g];
        if (s[g] < 1 || (dual[g] != 0 && dual[g] != 1) || H.n_edges < 0 || H.n_vertices < 0 ||
            (H.n_edges > 0 && !H.row_ptr)) {
            set_err(c, "invalid arguments for graph %s", std::to_string(g).c_str());
            return SLINE_EINVAL;
        }
    }
    std::unique_ptr<sline_batch_plan, void (*)(sline_batch_plan *)> P(new sline_batch_plan,
                                                                        plan_free);
    sline_batch_plan *p = P.get();
    p->c = c;
    p->G = G;
    p->flags = flags;
    p->weights = (flags & SLINE_NO_WEIGHTS) == 0;
    p->C.tune = c->tune;
    if (hipHostMalloc((void **)&p->host, sizeof(int64_t) * ((size_t)G + 17), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        p->host = nullptr;
        set_err(c, "batch plan: pinned host allocation failed");
        return SLINE_ENOMEM;
    }
    hipStream_t st = c->stream;
    // 1. descriptors and the graphs' nnz
    p->gr.resize(G);
    p->s_plan.assign(s, s + G);
    int32_t s_min = INT32_MAX;
    for (int32_t g = 0; g < G; ++g) {
        BatchGraph &d = p->gr[g];
        d = BatchGraph{};
        d.rp = Hs[g].row_ptr;
        d.col = Hs[g].col_idx;
        d.m = Hs[g].n_edges;
        d.n = Hs[g].n_vertices;
        d.dual = dual[g];
        d.s = s[g];
        s_min = std::min(s_min, s[g]);
    }
    p->s_min = G > 0 ? s_min : 1;
    {
        Arena W;
        const size_t small = sizeof(BatchGraph) * (size_t)std::max(G, 1) + 8 * (size_t)(5 * G + 16) + 4096;
        W.base = reinterpret_cast<char *>(plan_alloc(p, small, "descriptors"));
        p->d_gr = W.take<BatchGraph>(G);
        p->d_nnz = W.take<int64_t>(G);
        p->d_err = W.take<int32_t>(4);
        p->ibase = W.take<int64_t>(G + 1);
        p->off = W.take<int64_t>(G + 1);
        p->dbase = W.take<int64_t>(G + 1);
        p->dual_ids = W.take<int32_t>(G);
        p->zb = W.take<int32_t>(G + 1);
    }
    std::vector<int64_t> nnz(G, 0);
    if (G > 0) {
        hip_check(c, launch_fill_i32(st, p->d_err, 4, 0), "zero flags");
        hip_check(c, hipMemcpyAsync(p->d_gr, p->gr.data(), sizeof(BatchGraph) * G,
                                    hipMemcpyHostToDevice, st),
                  "upload graphs");
        hip_check(c, launch_batch_nnz(st, p->d_gr, G, p->d_nnz, p->d_err), "batch nnz");
        hip_check(c, hipMemcpyAsync(nnz.data(), p->d_nnz, sizeof(int64_t) * G,
                                    hipMemcpyDeviceToHost, st),
                  "read nnz");
        hip_check(c, hipMemcpyAsync(p->host, p->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read flags");
        sync(c, "batch nnz");
        if (reinterpret_cast<const int32_t *>(p->host)[0]) {
            set_err(c, "row_ptr must start at 0 in every graph");
            return SLINE_EINVAL;
        }
    }
    // 2. bases, combine and build arrays
    const sline_status rb = batch_bases(c, p->gr, nnz, p->B);
    if (rb != SLINE_OK) return rb;
    const BatchBases &B = p->B;
    p->C.tune = build_tuning(c->tune, B.NI);
    if (G > 0) {
        hip_check(c, hipMemcpyAsync(p->d_gr, p->gr.data(), sizeof(BatchGraph) * G,
                                    hipMemcpyHostToDevice, st),
                  "upload graphs");
        hip_check(c, hipMemcpyAsync(p->ibase, B.ibase.data(), sizeof(int64_t) * (G + 1),
                                    hipMemcpyHostToDevice, st),
                  "upload item bases");
        if (B.GD() > 0) {
            hip_check(c, hipMemcpyAsync(p->dbase, B.dbase.data(), sizeof(int64_t) * (B.GD() + 1),
                                        hipMemcpyHostToDevice, st),
                      "upload dual bases");
            hip_check(c, hipMemcpyAsync(p->dual_ids, B.dual_ids.data(), sizeof(int32_t) * B.GD(),
                                        hipMemcpyHostToDevice, st),
                      "upload dual ids");
        }
    }
    if (B.ZT > 0) {
        Arena sz;
        (void)plan_combine(sz, B);
        (void)plan_layout(sz, B.NI, B.MT, B.ZT, B.NI, B.MT, true);
        Arena A;
        A.base = reinterpret_cast<char *>(plan_alloc(p, sz.off + 4096, "the batch arrays"));
        p->K = plan_combine(A, B);
        p->L = plan_layout(A, B.NI, B.MT, B.ZT, B.NI, B.MT, true);
        p->C.ptrI = p->K.ptrC;
    }
    // 3. one run of the preparation, without guards: the task count
    if (G > 0) {
        plan_enqueue_prep(p, st, -1);
        int64_t *h = p->host;
        if (B.ZT > 0) {
            hip_check(c, hipMemcpyAsync(h + 0, p->L.tbase + B.NI, sizeof(int64_t),
                                        hipMemcpyDeviceToHost, st),
                      "read tasks");
            hip_check(c, hipMemcpyAsync(h + 1, p->L.totals, 3 * sizeof(int64_t),
                                        hipMemcpyDeviceToHost, st),
                      "read totals");
        }
        hip_check(c, hipMemcpyAsync(h + 4, p->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read flags");
        sync(c, "batch plan tasks");
        const int32_t e = reinterpret_cast<const int32_t *>(h + 4)[0];
        if (e) return plan_csr_error(c, e);
    }
    if (B.ZT > 0) {
        const int64_t T = p->host[0], wedges = p->host[3];
        if (T >= INT32_MAX) {
            set_err(c, "too many counting tasks (%s)", std::to_string(T).c_str());
            return SLINE_ENOMEM;
        }
        p->t_cap = std::max<int64_t>(T, 1);
        {
            Arena sz;
            (void)plan_tasks(sz, p->t_cap);
            Arena A;
            A.base = reinterpret_cast<char *>(plan_alloc(p, sz.off + 4096, "the task arrays"));
            p->TL = plan_tasks(A, p->t_cap);
        }
        // 4. one counting pass with a pool of W_s / s_min pairs (every pair
        // of L_s takes at least s wedges): the pair count
        plan_pool(p, wedges / p->s_min);
        void *first_pool = p->pool;
        p->C = plan_count_args(p);
        plan_enqueue_count(p, st, -1);
        int64_t *h = p->host;
        hip_check(c, hipMemcpyAsync(h + 0, p->TL.off + p->t_cap, sizeof(int64_t),
                                    hipMemcpyDeviceToHost, st),
                  "read pairs");
        hip_check(c, hipMemcpyAsync(h + 1, p->L.err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read flags");
        sync(c, "batch plan pairs");
        if (reinterpret_cast<const int32_t *>(h + 1)[0] & kErrInternal) {
            set_err(c, "internal error: counting table overflow");
            return SLINE_EDEVICE;
        }
        const int64_t total = h[0];
        p->pair_cap = std::max<int64_t>(total, 1);
        // the pool kept for the runs, instead of the W_s / s_min bound: a
        // range that does not fit its workgroup's chunk leaves less than its
        // own size unused, so the pairs take at most twice their number plus
        // the chunks left partly used at the end (one per workgroup, at most
        // an eighth of the pool in all); tasks that still find no room are
        // counted again by the fill pass
        const int64_t groups =
            (int64_t)c->n_cu * (p->C.tune.small_grid_per_cu + p->C.tune.task_grid_per_cu);
        const int64_t keep = std::min<int64_t>(p->pool_cap, total * 7 / 3 + 512 * groups);
        if (first_pool && keep < p->pool_cap) {
            plan_drop_last(p, first_pool);
            plan_pool(p, keep);
        }
        p->C = plan_count_args(p);
        const size_t bytes = sizeof(int32_t) * (size_t)p->pair_cap;
        p->out_a = reinterpret_cast<int32_t *>(plan_alloc(p, bytes, "the result arrays"));
        p->out_b = reinterpret_cast<int32_t *>(plan_alloc(p, bytes, "the result arrays"));
        if (p->weights)
            p->out_w = reinterpret_cast<int32_t *>(plan_alloc(p, bytes, "the result arrays"));
    }
    // 5. capture every stage, with the guards, on a stream of the plan's own
    // (the context's stream may be the null stream, which cannot capture)
    sync(c, "batch plan buffers");
    if (G == 0) {
        *out = P.release();
        return SLINE_OK;
    }
    hip_check(c, hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking), "capture stream");
    hip_check(c, hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
        plan_enqueue_prep(p, p->cap, p->t_cap);
        plan_enqueue_count(p, p->cap, p->pair_cap);
        plan_enqueue_fill(p, p->cap);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(p->cap, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        throw;
    }
    hip_check(c, hipStreamEndCapture(p->cap, &p->graph), "end capture");
    hip_check(c, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "graph instantiate");
    *out = P.release();
    return SLINE_OK;
}

sline_status plan_run_impl(sline_batch_plan *p, const int32_t *s, sline_edges *outs) {
    sline_ctx *c = p->c;
    const int32_t G = p->G;
    if (G > 0 && !outs) {
        set_err(c, "outs is NULL");
        return SLINE_EINVAL;
    }
    if (G == 0) return SLINE_OK;
    hipStream_t st = c->stream;
    // every s is checked before any is taken: a refused run leaves the
    // descriptors (host and device copies alike) as they were
    for (int32_t g = 0; s && g < G; ++g) {
        if (s[g] < p->s_plan[g]) {
            set_err(c, "batch plan: graph %s asks for an s below its planned s",
                    std::to_string(g).c_str());
            return SLINE_EINVAL;
        }
    }
    bool changed = p->gr_stale;
    for (int32_t g = 0; g < G; ++g) {
        const int32_t want = s ? s[g] : p->s_plan[g];
        changed = changed || want != p->gr[g].s;
        p->gr[g].s = want;
    }
    if (changed) {
        p->gr_stale = true;
        hip_check(c, hipMemcpyAsync(p->d_gr, p->gr.data(), sizeof(BatchGraph) * G,
                                    hipMemcpyHostToDevice, st),
                  "upload graphs");
        p->gr_stale = false;
    }
    hip_check(c, hipGraphLaunch(p->exec, st), "graph launch");
    int64_t *h = p->host;
    int64_t *w = h + G + 1;
    hip_check(c, hipMemcpyAsync(h, p->off, sizeof(int64_t) * (G + 1), hipMemcpyDeviceToHost, st),
              "read offsets");
    hip_check(c, hipMemcpyAsync(w, p->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
              "read flags");
    if (p->B.ZT > 0) {
        hip_check(c, hipMemcpyAsync(w + 1, p->L.err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read flags");
        hip_check(c, hipMemcpyAsync(w + 2, p->L.totals, 3 * sizeof(int64_t), hipMemcpyDeviceToHost,
                                    st),
                  "read totals");
        hip_check(c, hipMemcpyAsync(w + 5, p->L.passes, sizeof(int64_t), hipMemcpyDeviceToHost, st),
                  "read passes");
    } else {
        w[1] = 0;
    }
    sync(c, "batch plan run");
    const int32_t e = reinterpret_cast<const int32_t *>(w)[0];
    // a malformed input first: its counts mean nothing
    if (e & ~(kErrPlanTasks | kErrPlanPairs)) return plan_csr_error(c, e);
    if (e) {
        set_err(c, "batch plan: the run needs more %s than the plan holds; make a new plan",
                (e & kErrPlanTasks) ? "counting tasks" : "pairs");
        return SLINE_ECAPACITY;
    }
    if (reinterpret_cast<const int32_t *>(w + 1)[0] & kErrInternal) {
        set_err(c, "internal error: counting table overflow");
        return SLINE_EDEVICE;
    }
    if (h[0] != 0 || h[G] > p->pair_cap) {
        set_err(c, "internal error: graph pair offsets out of range");
        return SLINE_EDEVICE;
    }
    for (int32_t g = 0; g < G; ++g) {
        const int64_t n = h[g + 1] - h[g];
        if (n < 0) {
            set_err(c, "internal error: graph pair offsets out of order");
            return SLINE_EDEVICE;
        }
        sline_edges &o = outs[g];
        o.n_pairs = n;
        o.capacity = 0;
        o.a = p->out_a ? p->out_a + h[g] : nullptr;
        o.b = p->out_b ? p->out_b + h[g] : nullptr;
        o.w = p->out_w ? p->out_w + h[g] : nullptr;
    }
    sline_stats S{};
    S.n_items = p->B.NI;
    S.nnz = p->B.ZT;
    if (p->B.ZT > 0) {
        S.n_kept = w[2];
        S.nnz_kept = w[3];
        S.wedges = w[4];
        S.passes = w[5];
    }
    S.n_pairs = h[G];
    c->stats = S;
    return SLINE_OK;
}

// ------------------------------------------------------ SpGEMM companion

// L_s by the product route (Sec. IV-D): C = H H^T with both triangles and the
// diagonal, computed row by row (Gustavson) with the same LDS hash
// accumulators, materialized in full, then filtered to b > a, w >= s.  No
// degree pruning or lookup-only members: the product does not know s.
sline_status spgemm_impl(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual, uint32_t flags,
                         sline_edges *out) {
    if (flags & kBuildOnlyFlags) {
        set_err(c, "relabeling and the ablation flags apply to sline_build only");
        return SLINE_EINVAL;
    }
    if (!out) {
        set_err(c, "out is NULL");
        return SLINE_EINVAL;
    }
    if (s < 1 || (dual != 0 && dual != 1) || H.n_edges < 0 || H.n_vertices < 0) {
        set_err(c, "invalid argument (s >= 1, dual in {0,1}, sizes >= 0 required)");
        return SLINE_EINVAL;
    }
    if (out->capacity < 0 ||
        (out->capacity > 0 && (!out->a || !out->b || (!out->w && !(flags & SLINE_NO_WEIGHTS))))) {
        set_err(c, "output buffers: capacity > 0 requires a, b and (without SLINE_NO_WEIGHTS) w");
        return SLINE_EINVAL;
    }
    c->pending.valid = false;
    drop_batch_pending(c);
    release_pool(c);
    hipStream_t st = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    sline_edges P{};
    ItemS IS;
    IS.full = true;
    // the filter reads the product's weights whatever the caller asked for
    const sline_status r = build_core(c, H, 1, dual, flags & ~(uint32_t)SLINE_NO_WEIGHTS, &P, IS);
    release_pool(c);
    if (r != SLINE_OK) return r;
    sync(c, "product");
    auto t1 = std::chrono::steady_clock::now();
    const int64_t nP = P.n_pairs;
    const size_t pbytes = sizeof(int32_t) * (size_t)std::max<int64_t>(nP, 1);
    auto free_product = [&]() {
        if (P.a) {
            (void)hipStreamSynchronize(st);
            dev_free(c, P.a, pbytes);
            dev_free(c, P.b, pbytes);
            dev_free(c, P.w, pbytes);
        }
    };
    try {
        const int64_t tiles = (nP + kFilterTile - 1) / kFilterTile;
        int64_t total = 0;
        int32_t *cnt = nullptr;
        int64_t *off = nullptr, *part = nullptr;
        void *fw = nullptr;
        size_t fw_bytes = 0;
        if (tiles > 0) {
            Arena sz;
            sz.take<int32_t>(tiles);
            sz.take<int64_t>(tiles + 1);
            sz.take<int64_t>(scan_partials(tiles + 1));
            fw_bytes = sz.off + 4096;
            fw = dev_alloc(c, fw_bytes);
            if (!fw) {
                set_err(c, "filter workspace allocation failed");
                throw Fail{SLINE_ENOMEM};
            }
            Arena A;
            A.base = reinterpret_cast<char *>(fw);
            cnt = A.take<int32_t>(tiles);
            off = A.take<int64_t>(tiles + 1);
            part = A.take<int64_t>(scan_partials(tiles + 1));
            hip_check(c, launch_product_filter(st, P.a, P.b, P.w, nP, s, cnt, nullptr, nullptr, nullptr,
                                               nullptr),
                      "product filter count");
            hip_check(c, launch_scan_i32_to_i64(st, cnt, tiles, off, part), "product filter scan");
            hip_check(c, hipMemcpyAsync(c->host, off + tiles, sizeof(int64_t), hipMemcpyDeviceToHost, st),
                      "read filtered size");
            sync(c, "product filter count");
            total = c->host[0];
        }
        if (out->capacity > 0 && out->capacity < total) {
            out->n_pairs = total;
            if (fw) dev_free(c, fw, fw_bytes);
            free_product();
            set_err(c, "capacity too small");
            return SLINE_ECAPACITY;
        }
        int32_t *a = out->a, *b = out->b;
        int32_t *w = (flags & SLINE_NO_WEIGHTS) ? nullptr : out->w;
        bool owned = false;
        if (out->capacity == 0) {
            a = b = w = nullptr;
            if (total > 0) {
                const size_t bytes = sizeof(int32_t) * (size_t)total;
                a = (int32_t *)dev_alloc(c, bytes);
                b = (int32_t *)dev_alloc(c, bytes);
                w = (flags & SLINE_NO_WEIGHTS) ? nullptr : (int32_t *)dev_alloc(c, bytes);
                owned = true;
                if (!a || !b || (!w && !(flags & SLINE_NO_WEIGHTS))) {
                    dev_free(c, a, bytes);
                    dev_free(c, b, bytes);
                    dev_free(c, w, bytes);
                    set_err(c, "output allocation failed");
                    throw Fail{SLINE_ENOMEM};
                }
            }
        }
        if (total > 0)
            hip_check(c, launch_product_filter(st, P.a, P.b, P.w, nP, s, cnt, off, a, b, w),
                      "product filter write");
        sync(c, "product filter");
        if (fw) dev_free(c, fw, fw_bytes);
        (void)owned;
        if (out->capacity == 0) {
            out->a = a;
            out->b = b;
            out->w = w;
        }
        out->n_pairs = total;
    } catch (...) {
        free_product();
        throw;
    }
    free_product();
    auto t2 = std::chrono::steady_clock::now();
    c->stats.product_nnz = nP;
    c->stats.n_pairs = out->n_pairs;
    c->stats.ms_product = std::chrono::duration<double, std::milli>(t1 - t0).count();
    c->stats.ms_filter = std::chrono::duration<double, std::milli>(t2 - t1).count();
    return SLINE_OK;
}

}  // namespace

// ------------------------------------------------ stages after L_s, variants

namespace {

constexpr uint32_t kRelabelFlags = SLINE_RELABEL_DESC | SLINE_RELABEL_ASC;

// One device block for the temporaries of a call, carved by an Arena and
// released (after the stream is idle) when the call leaves.
struct TempBlock {
    sline_ctx *c;
    void *p = nullptr;
    size_t bytes = 0;
    explicit TempBlock(sline_ctx *cc) : c(cc) {}
    char *get(size_t n, const char *what) {
        bytes = n + 4096;
        p = dev_alloc(c, bytes);
        if (!p) {
            set_err(c, "allocation of temporaries failed (%s)", what);
            throw Fail{SLINE_ENOMEM};
        }
        return static_cast<char *>(p);
    }
    ~TempBlock() {
        if (p) {
            (void)hipStreamSynchronize(c->stream);
            dev_free(c, p, bytes);
        }
    }
};

// Device arrays of an edge list the library allocated, freed on scope exit
// unless released.
struct OwnedEdges {
    sline_ctx *c;
    sline_edges e{};
    explicit OwnedEdges(sline_ctx *cc) : c(cc) {}
    void alloc(int64_t n, bool weights, const char *what) {
        const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1);
        e.n_pairs = n;
        e.a = (int32_t *)dev_alloc(c, bytes);
        e.b = e.a ? (int32_t *)dev_alloc(c, bytes) : nullptr;
        e.w = (e.b && weights) ? (int32_t *)dev_alloc(c, bytes) : nullptr;
        if (!e.a || !e.b || (weights && !e.w)) {
            set_err(c, "allocation of %s failed", what);
            throw Fail{SLINE_ENOMEM};
        }
    }
    sline_edges release() {
        sline_edges r = e;
        e = sline_edges{};
        return r;
    }
    ~OwnedEdges() {
        if (e.a || e.b || e.w) {
            (void)hipStreamSynchronize(c->stream);
            const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(e.n_pairs, 1);
            dev_free(c, e.a, bytes);
            dev_free(c, e.b, bytes);
            dev_free(c, e.w, bytes);
        }
    }
};

// Buffers of one radix-sort transpose over n entries with keys in [0, nk).
struct SortBufs {
    int32_t *rsK[2], *rsV[2], *hist, *part32, *ptrT;
};

SortBufs plan_sort(Arena &A, int64_t n, int64_t nk) {
    SortBufs B{};
    B.rsK[0] = A.take<int32_t>(n);
    B.rsK[1] = A.take<int32_t>(n);
    B.rsV[0] = A.take<int32_t>(n);
    B.rsV[1] = A.take<int32_t>(n);
    B.hist = A.take<int32_t>(transpose_hist(n));
    // partials of the digit scans, and of scans over n or nk entries
    B.part32 = A.take<int32_t>(
        scan_partials(std::max<int64_t>({transpose_hist(n), nk, n}) + 1));
    B.ptrT = A.take<int32_t>(nk + 1);
    return B;
}

// Pairs (a, b, w) into (a, b) order: a stable radix sort by b, then a stable
// one by a, both through the transpose (ids in [0, nk), n < 2^31).  oa, ob,
// ow receive the result (ow and w may be null).  Writes a1..k2 scratch.
void sort_pairs(sline_ctx *c, const int32_t *a, const int32_t *b, const int32_t *w, int64_t n,
                int32_t nk, int32_t *oa, int32_t *ob, int32_t *ow) {
    if (n <= 0) return;
    hipStream_t st = c->stream;
    auto plan = [&](Arena &A, SortBufs &B, int32_t *&a1, int32_t *&b1, int32_t *&k1,
                    int32_t *&w1, int32_t *&k2) {
        B = plan_sort(A, n, nk);
        a1 = A.take<int32_t>(n);
        b1 = A.take<int32_t>(n);
        k1 = A.take<int32_t>(n);
        w1 = w ? A.take<int32_t>(n) : nullptr;
        k2 = A.take<int32_t>(n);
    };
    SortBufs B;
    int32_t *a1, *b1, *k1, *w1, *k2;
    Arena sz;
    plan(sz, B, a1, b1, k1, w1, k2);
    TempBlock T(c);
    Arena A;
    A.base = T.get(sz.off, "pair sort");
    plan(A, B, a1, b1, k1, w1, k2);
    const int last = (transpose_passes(nk) - 1) & 1;
    // by b: a1 = the a of each pair in b order, its sorted b in rsK[last]
    hip_check(c, launch_transpose(st, b, n, nk, a, B.rsK, B.rsV, B.hist, B.part32, B.ptrT, a1, k1,
                                  nullptr),
              "pair sort (second key)");
    hip_check(c, launch_copy_i32(st, b1, B.rsK[last], n), "pair sort copy");
    if (w) hip_check(c, launch_gather(st, w, k1, n, w1), "pair sort gather");
    // by a, stable: ties keep b order
    hip_check(c, launch_transpose(st, a1, n, nk, b1, B.rsK, B.rsV, B.hist, B.part32, B.ptrT, ob, k2,
                                  nullptr),
              "pair sort (first key)");
    hip_check(c, launch_copy_i32(st, oa, B.rsK[last], n), "pair sort copy");
    if (w && ow) hip_check(c, launch_gather(st, w1, k2, n, ow), "pair sort gather");
    sync(c, "pair sort");
}

// Hand a computed edge list (library-owned arrays `res`, n pairs) to the
// caller's `out` under the capacity protocol: moved when out->capacity is 0,
// copied into caller buffers otherwise (SLINE_ECAPACITY if too small).
sline_status deliver(sline_ctx *c, OwnedEdges &res, sline_edges *out, bool weights) {
    const int64_t n = res.e.n_pairs;
    if (out->capacity > 0 && out->capacity < n) {
        out->n_pairs = n;
        set_err(c, "capacity too small");
        return SLINE_ECAPACITY;
    }
    if (out->capacity == 0) {
        if (n == 0) {
            out->n_pairs = 0;
            out->a = out->b = out->w = nullptr;
            return SLINE_OK;
        }
        const sline_edges r = res.release();
        out->n_pairs = n;
        out->a = r.a;
        out->b = r.b;
        out->w = weights ? r.w : nullptr;
        if (!weights && r.w) dev_free(c, r.w, sizeof(int32_t) * (size_t)n);
        return SLINE_OK;
    }
    hipStream_t st = c->stream;
    hip_check(c, launch_copy_i32(st, out->a, res.e.a, n), "copy result");
    hip_check(c, launch_copy_i32(st, out->b, res.e.b, n), "copy result");
    if (weights && out->w && res.e.w) hip_check(c, launch_copy_i32(st, out->w, res.e.w, n), "copy result");
    sync(c, "copy result");
    out->n_pairs = n;
    return SLINE_OK;
}

// The CSR rules of sline_csr, checked on the device; returns nnz.
int64_t validate_csr(sline_ctx *c, const sline_csr &H, uint32_t flags) {
    hipStream_t st = c->stream;
    const int64_t m = H.n_edges, n = H.n_vertices;
    if (m > 0 && !H.row_ptr) {
        set_err(c, "row_ptr is NULL");
        throw Fail{SLINE_EINVAL};
    }
    TempBlock T0(c);
    int32_t *err = reinterpret_cast<int32_t *>(T0.get(64, "flags"));
    hip_check(c, launch_fill_i32(st, err, 4, 0), "zero flags");
    int32_t *h = reinterpret_cast<int32_t *>(c->host);
    h[0] = 0;
    if (m > 0) {
        hip_check(c, launch_check_rowptr(st, H.row_ptr, (int32_t)m, err), "row_ptr check");
        hip_check(c, hipMemcpyAsync(h, H.row_ptr + m, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read nnz");
    }
    hip_check(c, hipMemcpyAsync(h + 1, err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read flags");
    sync(c, "row_ptr check");
    const int64_t nnz = h[0];
    if (h[1] != 0 || nnz < 0) {
        set_err(c, "row_ptr must start at 0 and never decrease");
        throw Fail{SLINE_EINVAL};
    }
    if (nnz > 0 && (!H.col_idx || n == 0)) {
        set_err(c, "col_idx is NULL or n_vertices is 0 with nnz > 0");
        throw Fail{SLINE_EINVAL};
    }
    if (nnz > 0) {
        TempBlock T1(c);
        int32_t *rowid = reinterpret_cast<int32_t *>(T1.get(sizeof(int32_t) * (size_t)nnz, "row ids"));
        hip_check(c, launch_rows(st, H.row_ptr, H.col_idx, (int32_t)m, (int32_t)n, nnz,
                                 (flags & SLINE_SKIP_VALIDATE) ? 0 : 1, rowid, err),
                  "row check");
        hip_check(c, hipMemcpyAsync(h + 1, err, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "read flags");
        sync(c, "row check");
        if (h[1] & (kErrColRange | kErrColOrder)) {
            set_err(c, "col_idx: members must lie in [0, n_vertices) and increase strictly within a row");
            throw Fail{SLINE_EINVAL};
        }
    }
    return nnz;
}

// sline_build with SLINE_RELABEL_*: renumber the side's items by size, build,
// map the pairs back and sort them (Sec. IV-F).
sline_status relabel_impl(sline_ctx *c, const sline_csr &H, int32_t s, int32_t dual,
                          uint32_t flags, sline_edges *out) {
    const bool desc = (flags & SLINE_RELABEL_DESC) != 0;
    if ((flags & kRelabelFlags) == kRelabelFlags) {
        set_err(c, "SLINE_RELABEL_DESC and SLINE_RELABEL_ASC exclude each other");
        return SLINE_EINVAL;
    }
    const int64_t nnz = validate_csr(c, H, flags);
    hipStream_t st = c->stream;
    const int32_t m = H.n_edges, n = H.n_vertices;
    const int32_t N = dual ? n : m;
    const bool weights = !(flags & SLINE_NO_WEIGHTS);
    // 1. sizes, the permutation (stable by size, ties by id) and its inverse
    Arena sz;
    auto plan = [&](Arena &A, int32_t *&size, int32_t *&mx, int32_t *&key, int32_t *&ids,
                    int32_t *&perm, int32_t *&inv, SortBufs &B, int32_t *&ptrV, int32_t *&colV,
                    SortBufs &BV) {
        size = A.take<int32_t>(N);
        mx = A.take<int32_t>(4);
        key = A.take<int32_t>(N);
        ids = A.take<int32_t>(N);
        perm = A.take<int32_t>(N);
        inv = A.take<int32_t>(N);
        // sizes are at most max(nnz, 1); the key sort spans that many buckets
        B = plan_sort(A, N, std::max<int64_t>(nnz, 1) + 1);
        ptrV = nullptr;
        colV = nullptr;
        if (dual) {  // vertex degrees from the transpose of H
            BV = plan_sort(A, std::max<int64_t>(nnz, 1), n);
            ptrV = BV.ptrT;
            colV = A.take<int32_t>(std::max<int64_t>(nnz, 1));
        }
    };
    int32_t *size, *mx, *key, *ids, *perm, *inv, *ptrV, *colV;
    SortBufs B{}, BV{};
    plan(sz, size, mx, key, ids, perm, inv, B, ptrV, colV, BV);
    TempBlock T(c);
    Arena A;
    A.base = T.get(sz.off, "relabel");
    plan(A, size, mx, key, ids, perm, inv, B, ptrV, colV, BV);
    hip_check(c, launch_fill_i32(st, mx, 4, 0), "zero max");
    const int32_t *item_ptr = H.row_ptr;
    if (dual) {
        TempBlock TR(c);
        int32_t *rowid = reinterpret_cast<int32_t *>(TR.get(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1), "row ids"));
        hip_check(c, launch_row_ids(st, H.row_ptr, m, rowid), "row ids");
        hip_check(c, launch_transpose(st, H.col_idx, nnz, n, rowid, BV.rsK, BV.rsV, BV.hist, BV.part32,
                                      BV.ptrT, colV, nullptr, nullptr),
                  "vertex lists");
        item_ptr = ptrV;
        sync(c, "vertex lists");
    }
    hip_check(c, launch_sizes(st, item_ptr, N, size, mx), "item sizes");
    hip_check(c, hipMemcpyAsync(c->host, mx, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read max size");
    sync(c, "item sizes");
    const int32_t max_size = reinterpret_cast<const int32_t *>(c->host)[0];
    hip_check(c, launch_size_keys(st, size, N, mx, desc ? 1 : 0, key), "size keys");
    hip_check(c, launch_iota(st, ids, N), "ids");
    if (N > 0)
        hip_check(c, launch_transpose(st, key, N, max_size + 1, ids, B.rsK, B.rsV, B.hist, B.part32,
                                      B.ptrT, perm, nullptr, nullptr),
                  "size order");
    hip_check(c, launch_invert(st, perm, N, inv), "inverse order");
    // 2. the renumbered hypergraph
    TempBlock TH(c);
    sline_csr H2 = H;
    {
        Arena hs;
        hs.take<int32_t>((int64_t)m + 1);
        hs.take<int32_t>(std::max<int64_t>(nnz, 1));
        hs.take<int32_t>(std::max<int64_t>(N, 1));
        hs.take<int32_t>(std::max<int64_t>(nnz, 1));
        hs.take<int32_t>(std::max<int64_t>(nnz, 1));
        hs.take<int32_t>(std::max<int64_t>(nnz, 1));
        Arena ha;
        ha.base = TH.get(hs.off, "relabeled hypergraph");
        int32_t *nrp = ha.take<int32_t>((int64_t)m + 1);
        int32_t *ncol = ha.take<int32_t>(std::max<int64_t>(nnz, 1));
        int32_t *len = ha.take<int32_t>(std::max<int64_t>(N, 1));
        int32_t *rowid = ha.take<int32_t>(std::max<int64_t>(nnz, 1));
        int32_t *rcol = ha.take<int32_t>(std::max<int64_t>(nnz, 1));
        int32_t *rrow = ha.take<int32_t>(std::max<int64_t>(nnz, 1));
        if (!dual) {
            // rows in the new order
            hip_check(c, launch_perm_rows(st, H.row_ptr, H.col_idx, perm, m, len, nrp, B.part32, ncol),
                      "relabeled rows");
            H2.row_ptr = nrp;
            H2.col_idx = ncol;
        } else if (nnz > 0) {
            // vertex ids renumbered, every row sorted again
            hip_check(c, launch_row_ids(st, H.row_ptr, m, rowid), "row ids");
            hip_check(c, launch_gather(st, inv, H.col_idx, nnz, rcol), "renumbered members");
            sort_pairs(c, rowid, rcol, nullptr, nnz, std::max(m, n), rrow, ncol, nullptr);
            H2.col_idx = ncol;
        }
        sync(c, "relabeled hypergraph");
        // 3. build on it, 4. map back and sort
        OwnedEdges tmp(c);
        ItemS IS;
        IS.s_min = IS.s_max = s;
        sline_edges t{};
        const sline_status r = build_core(c, H2, s, dual, (flags & ~kRelabelFlags) | SLINE_SKIP_VALIDATE,
                                          &t, IS);
        tmp.e = t;
        if (r != SLINE_OK) return r;
        const int64_t np = t.n_pairs;
        if (np >= INT32_MAX) {
            set_err(c, "relabeled builds handle results below 2^31 pairs");
            return SLINE_EINVAL;
        }
        OwnedEdges res(c);
        res.alloc(np, weights, "relabeled result");
        if (np > 0) {
            TempBlock TM(c);
            Arena ms;
            ms.take<int32_t>(np);
            ms.take<int32_t>(np);
            Arena ma;
            ma.base = TM.get(ms.off, "mapped pairs");
            int32_t *x = ma.take<int32_t>(np);
            int32_t *y = ma.take<int32_t>(np);
            hip_check(c, launch_map_pairs(st, t.a, t.b, np, perm, x, y), "map back");
            sort_pairs(c, x, y, weights ? t.w : nullptr, np, N, res.e.a, res.e.b,
                       weights ? res.e.w : nullptr);
        }
        const sline_stats keep = c->stats;
        const sline_status d = deliver(c, res, out, weights);
        c->stats = keep;
        return d;
    }
}

// sline_build with SLINE_NO_VISITED: one set intersection per wedge, the
// accepted pairs written per item in any order, then sorted.  Called by
// build_core once the member lists, back-pointers and costs are ready.
sline_status intersect_build(sline_ctx *c, const int32_t *ptrI, const int32_t *memI,
                             const int32_t *ptrS, const int32_t *itmS, const int32_t *start,
                             int32_t N, int32_t s, uint32_t flags, int32_t *cnt, int64_t *off,
                             int64_t *part64, unsigned long long *inters, sline_edges *out,
                             sline_stats &S) {
    hipStream_t st = c->stream;
    const bool prune = !(flags & SLINE_NO_PRUNE);
    const bool shortcut = !(flags & SLINE_NO_SHORTCUT);
    const bool weights = !(flags & SLINE_NO_WEIGHTS);
    hip_check(c, launch_fill_i32(st, cnt, N, 0), "zero counts");
    mark(c, 2);
    hip_check(c, launch_wedge_intersect(st, ptrI, memI, ptrS, itmS, start, N, s, prune ? 1 : 0,
                                        shortcut ? 1 : 0, cnt, nullptr, nullptr, nullptr, nullptr,
                                        inters, c->n_cu),
              "intersections (count)");
    hip_check(c, launch_scan_i32_to_i64(st, cnt, N, off, part64), "pair scan");
    mark(c, 3);
    int64_t *h = c->host;
    hip_check(c, hipMemcpyAsync(h, off + N, sizeof(int64_t), hipMemcpyDeviceToHost, st), "read total");
    hip_check(c, hipMemcpyAsync(h + 1, inters, sizeof(int64_t), hipMemcpyDeviceToHost, st),
              "read intersections");
    sync(c, "intersections");
    const int64_t total = h[0];
    S.intersections = h[1];
    S.n_pairs = total;
    if (c->profile) S.ms_count = span_ms(c, 2, 3);
    c->stats = S;
    if (total >= INT32_MAX) {
        set_err(c, "builds without visited skipping handle results below 2^31 pairs");
        return SLINE_EINVAL;
    }
    if (out->capacity > 0 && out->capacity < total) {
        out->n_pairs = total;
        set_err(c, "capacity too small");
        return SLINE_ECAPACITY;
    }
    OwnedEdges raw(c), res(c);
    raw.alloc(total, true, "unsorted pairs");
    res.alloc(total, weights, "result");
    mark(c, 5);
    if (total > 0) {
        hip_check(c, launch_wedge_intersect(st, ptrI, memI, ptrS, itmS, start, N, s, prune ? 1 : 0,
                                            shortcut ? 1 : 0, cnt, off, raw.e.a, raw.e.b, raw.e.w,
                                            nullptr, c->n_cu),
                  "intersections (write)");
        sort_pairs(c, raw.e.a, raw.e.b, raw.e.w, total, N, res.e.a, res.e.b,
                   weights ? res.e.w : nullptr);
    }
    mark(c, 6);
    sync(c, "intersections");
    if (c->profile) S.ms_fill = span_ms(c, 5, 6);
    c->stats = S;
    return deliver(c, res, out, weights);
}

sline_status filter_impl(sline_ctx *c, const sline_edges *in, int32_t s, uint32_t flags,
                         sline_edges *out) {
    if (!in || !out || s < 1 || in->n_pairs < 0 ||
        (in->n_pairs > 0 && (!in->a || !in->b || !in->w))) {
        set_err(c, "invalid arguments (s >= 1 and an input with a, b and w required)");
        return SLINE_EINVAL;
    }
    if (out->capacity < 0 ||
        (out->capacity > 0 && (!out->a || !out->b || (!out->w && !(flags & SLINE_NO_WEIGHTS))))) {
        set_err(c, "output buffers: capacity > 0 requires a, b and (without SLINE_NO_WEIGHTS) w");
        return SLINE_EINVAL;
    }
    c->pending.valid = false;
    hipStream_t st = c->stream;
    const int64_t n = in->n_pairs;
    const bool weights = !(flags & SLINE_NO_WEIGHTS);
    const int64_t tiles = wfilter_tiles(n);
    int64_t total = 0;
    TempBlock T(c);
    int32_t *cnt = nullptr;
    int64_t *off = nullptr;
    if (n > 0) {
        Arena sz;
        sz.take<int32_t>(tiles);
        sz.take<int64_t>(tiles + 1);
        sz.take<int64_t>(scan_partials(tiles + 1));
        Arena A;
        A.base = T.get(sz.off, "filter");
        cnt = A.take<int32_t>(tiles);
        off = A.take<int64_t>(tiles + 1);
        int64_t *part = A.take<int64_t>(scan_partials(tiles + 1));
        hip_check(c, launch_wfilter(st, in->a, in->b, in->w, n, s, cnt, nullptr, nullptr, nullptr,
                                    nullptr),
                  "filter count");
        hip_check(c, launch_scan_i32_to_i64(st, cnt, tiles, off, part), "filter scan");
        hip_check(c, hipMemcpyAsync(c->host, off + tiles, sizeof(int64_t), hipMemcpyDeviceToHost, st),
                  "read filtered size");
        sync(c, "filter count");
        total = c->host[0];
    }
    if (out->capacity > 0 && out->capacity < total) {
        out->n_pairs = total;
        set_err(c, "capacity too small");
        return SLINE_ECAPACITY;
    }
    OwnedEdges res(c);
    int32_t *oa = out->a, *ob = out->b, *ow = weights ? out->w : nullptr;
    if (out->capacity == 0 && total > 0) {
        res.alloc(total, weights, "filtered pairs");
        oa = res.e.a;
        ob = res.e.b;
        ow = res.e.w;
    }
    if (total > 0) {
        hip_check(c, launch_wfilter(st, in->a, in->b, in->w, n, s, cnt, off, oa, ob, ow),
                  "filter write");
        sync(c, "filter write");
    }
    if (out->capacity == 0) {
        const sline_edges r = res.release();
        out->a = total ? r.a : nullptr;
        out->b = total ? r.b : nullptr;
        out->w = total ? r.w : nullptr;
    }
    out->n_pairs = total;
    return SLINE_OK;
}

sline_status sweep_impl(sline_ctx *c, const sline_csr &H, int32_t n_s, const int32_t *s_list,
                        int32_t dual, uint32_t flags, sline_edges *outs) {
    if (n_s < 0 || (n_s > 0 && (!s_list || !outs)) || (dual != 0 && dual != 1) ||
        (flags & SLINE_NO_WEIGHTS)) {
        set_err(c, "invalid sweep arguments (s_list and outs of n_s entries; no SLINE_NO_WEIGHTS)");
        return SLINE_EINVAL;
    }
    for (int32_t i = 0; i < n_s; ++i) {
        if (s_list[i] < 1 || outs[i].capacity != 0) {
            set_err(c, "every s >= 1, every output with capacity 0");
            return SLINE_EINVAL;
        }
    }
    if (n_s == 0) return SLINE_OK;
    std::vector<int32_t> order(n_s);
    for (int32_t i = 0; i < n_s; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return s_list[x] < s_list[y]; });
    std::vector<sline_edges> res(n_s);
    auto release_all = [&]() {
        for (auto &e : res) {
            if (e.a || e.b || e.w) (void)sline_edges_free(c, &e);
        }
    };
    sline_status r = build_impl(c, H, s_list[order[0]], dual, flags, &res[order[0]]);
    if (r != SLINE_OK) return r;
    try {
        for (int32_t k = 1; k < n_s; ++k) {
            const sline_edges &prev = res[order[k - 1]];
            r = filter_impl(c, &prev, s_list[order[k]], flags, &res[order[k]]);
            if (r != SLINE_OK) {
                release_all();
                return r;
            }
        }
    } catch (...) {
        release_all();
        throw;
    }
    for (int32_t i = 0; i < n_s; ++i) outs[i] = res[i];
    return SLINE_OK;
}

sline_status squeeze_impl(sline_ctx *c, int32_t N, const sline_edges *L, uint32_t flags,
                          sline_graph *G) {
    const bool weights = !(flags & SLINE_NO_WEIGHTS);
    if (!L || !G || N < 0 || L->n_pairs < 0 || L->n_pairs >= INT32_MAX ||
        (L->n_pairs > 0 && (!L->a || !L->b || (weights && !L->w)))) {
        set_err(c, "invalid arguments (pairs with a, b and w unless SLINE_NO_WEIGHTS; "
                   "n_pairs below 2^31)");
        return SLINE_EINVAL;
    }
    hipStream_t st = c->stream;
    const int64_t n = L->n_pairs;
    sline_graph g{};
    auto plan = [&](Arena &A, int32_t *&err, int32_t *&flag, int32_t *&newid, int32_t *&p32,
                    int64_t *&fwd, int32_t *&deg, int64_t *&off, int64_t *&p64, SortBufs &B,
                    int32_t *&colT, int32_t *&kT) {
        err = A.take<int32_t>(4);
        flag = A.take<int32_t>((int64_t)N + 1);
        newid = A.take<int32_t>((int64_t)N + 1);
        p32 = A.take<int32_t>(scan_partials((int64_t)N + 1));
        fwd = A.take<int64_t>((int64_t)N + 1);
        deg = A.take<int32_t>((int64_t)N + 1);
        off = A.take<int64_t>((int64_t)N + 1);
        p64 = A.take<int64_t>(scan_partials((int64_t)N + 1));
        B = plan_sort(A, std::max<int64_t>(n, 1), N);
        colT = A.take<int32_t>(std::max<int64_t>(n, 1));
        kT = A.take<int32_t>(std::max<int64_t>(n, 1));
    };
    int32_t *err, *flag, *newid, *p32, *deg, *colT, *kT;
    int64_t *fwd, *off, *p64;
    SortBufs B{};
    Arena sz;
    plan(sz, err, flag, newid, p32, fwd, deg, off, p64, B, colT, kT);
    TempBlock T(c);
    Arena A;
    A.base = T.get(sz.off, "squeeze");
    plan(A, err, flag, newid, p32, fwd, deg, off, p64, B, colT, kT);
    hip_check(c, launch_fill_i32(st, err, 4, 0), "zero flags");
    hip_check(c, launch_fill_i32(st, flag, (int64_t)N + 1, 0), "zero flags");
    // 1. items present (and the pairs checked: ids in range, a < b, sorted)
    hip_check(c, launch_mark_present(st, L->a, L->b, n, N, flag, err), "items present");
    hip_check(c, hipMemcpyAsync(c->host, err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read flags");
    sync(c, "items present");
    if (reinterpret_cast<const int32_t *>(c->host)[0]) {
        set_err(c, "pairs must have 0 <= a < b < n_items and be sorted by (a, b)");
        return SLINE_EINVAL;
    }
    // 2. new ids: exclusive scan of the presence flags
    hip_check(c, launch_scan_i32(st, flag, N, newid, p32), "new ids");
    hip_check(c, hipMemcpyAsync(c->host, newid + N, sizeof(int32_t), hipMemcpyDeviceToHost, st),
              "read node count");
    sync(c, "new ids");
    g.n_nodes = reinterpret_cast<const int32_t *>(c->host)[0];
    g.n_arcs = 2 * n;
    auto free_graph = [&]() {
        (void)hipStreamSynchronize(st);
        dev_free(c, g.old_id, sizeof(int32_t) * (size_t)std::max(g.n_nodes, 1));
        dev_free(c, g.row_ptr, sizeof(int64_t) * ((size_t)g.n_nodes + 1));
        dev_free(c, g.col, sizeof(int32_t) * (size_t)std::max<int64_t>(g.n_arcs, 1));
        dev_free(c, g.w, sizeof(int32_t) * (size_t)std::max<int64_t>(g.n_arcs, 1));
    };
    try {
        g.old_id = (int32_t *)dev_alloc(c, sizeof(int32_t) * (size_t)std::max(g.n_nodes, 1));
        g.row_ptr = (int64_t *)dev_alloc(c, sizeof(int64_t) * ((size_t)g.n_nodes + 1));
        g.col = (int32_t *)dev_alloc(c, sizeof(int32_t) * (size_t)std::max<int64_t>(g.n_arcs, 1));
        g.w = weights ? (int32_t *)dev_alloc(c, sizeof(int32_t) * (size_t)std::max<int64_t>(g.n_arcs, 1))
                      : nullptr;
        if (!g.old_id || !g.row_ptr || !g.col || (weights && !g.w)) {
            set_err(c, "graph allocation failed");
            throw Fail{SLINE_ENOMEM};
        }
        hip_check(c, launch_old_ids(st, flag, newid, N, g.old_id), "old ids");
        // 3. the pairs by second item (transpose), by first item (runs)
        hip_check(c, launch_transpose(st, L->b, n, N, L->a, B.rsK, B.rsV, B.hist, B.part32, B.ptrT,
                                      colT, kT, nullptr),
                  "pairs by second item");
        hip_check(c, launch_run_starts(st, L->a, n, N, fwd), "pairs by first item");
        // 4. degrees, row pointers, rows
        hip_check(c, launch_degrees(st, fwd, B.ptrT, N, deg), "degrees");
        hip_check(c, launch_scan_i32_to_i64(st, deg, N, off, p64), "row offsets");
        hip_check(c, launch_row_ptr(st, flag, newid, off, N, g.n_nodes, g.row_ptr), "row pointers");
        hip_check(c, launch_adj_fill(st, N, flag, newid, off, B.ptrT, colT, kT, fwd, L->b,
                                     weights ? L->w : nullptr, g.col, g.w),
                  "adjacency");
        sync(c, "adjacency");
    } catch (...) {
        free_graph();
        throw;
    }
    *G = g;
    return SLINE_OK;
}

sline_status components_impl(sline_ctx *c, int32_t N, const sline_edges *L, int32_t *comp,
                             int64_t *n_components) {
    if (!L || N < 0 || L->n_pairs < 0 || (N > 0 && !comp) ||
        (L->n_pairs > 0 && (!L->a || !L->b))) {
        set_err(c, "invalid arguments");
        return SLINE_EINVAL;
    }
    hipStream_t st = c->stream;
    const int64_t n = L->n_pairs;
    TempBlock T(c);
    Arena sz;
    sz.take<int32_t>(4);
    sz.take<unsigned long long>(1);
    sz.take<int32_t>((int64_t)N + 1);
    Arena A;
    A.base = T.get(sz.off, "components");
    int32_t *err = A.take<int32_t>(4);
    unsigned long long *count = A.take<unsigned long long>(1);
    int32_t *flag = A.take<int32_t>((int64_t)N + 1);
    hip_check(c, launch_fill_i32(st, err, 4, 0), "zero flags");
    hip_check(c, launch_fill_i64(st, reinterpret_cast<int64_t *>(count), 1, 0), "zero count");
    hip_check(c, launch_fill_i32(st, flag, (int64_t)N + 1, 0), "zero flags");
    hip_check(c, launch_mark_present(st, L->a, L->b, n, N, flag, err), "items present");
    hip_check(c, hipMemcpyAsync(c->host, err, sizeof(int32_t), hipMemcpyDeviceToHost, st), "read flags");
    sync(c, "items present");
    if (reinterpret_cast<const int32_t *>(c->host)[0]) {
        set_err(c, "pairs must have 0 <= a < b < n_items and be sorted by (a, b)");
        return SLINE_EINVAL;
    }
    hip_check(c, launch_components(st, L->a, L->b, n, N, comp), "components");
    hip_check(c, launch_cc_count(st, comp, flag, N, count), "component count");
    hip_check(c, hipMemcpyAsync(c->host, count, sizeof(int64_t), hipMemcpyDeviceToHost, st),
              "read component count");
    sync(c, "components");
    if (n_components) *n_components = c->host[0];
    return SLINE_OK;
}

// Entry-point wrapper: device, error capture.
template <typename F>
sline_status guarded(sline_ctx *c, F &&f) {
    if (!c) return SLINE_EINVAL;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return f();
    } catch (const Fail &fl) {
        c->pending.valid = false;
        release_pool(c);
        return fl.st;
    } catch (const std::bad_alloc &) {
        c->pending.valid = false;
        release_pool(c);
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

}  // namespace

extern "C" {

sline_status sline_create(sline_ctx **ctx, int device, void *hip_stream, const sline_allocator *alloc) {
    if (!ctx) return SLINE_EINVAL;
    *ctx = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return SLINE_EINVAL;
    sline_ctx *c = new (std::nothrow) sline_ctx();
    if (!c) return SLINE_ENOMEM;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (alloc) {
        c->alloc = *alloc;
        c->has_alloc = true;
    }
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SLINE_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->n_cu = ncu;
    // set-up of sline_build_noalloc: this device's address of the scratch
    // array (a failure is reported by that entry point, not here)
    (void)scratch_address(device);
    if (hipHostMalloc((void **)&c->host, 64 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SLINE_EDEVICE;
    }
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            sline_destroy(c);
            return SLINE_EDEVICE;
        }
    }
    *ctx = c;
    return SLINE_OK;
}

void sline_destroy(sline_ctx *c) {
    if (!c) return;
    release_pool(c);
    drop_batch_pending(c);
    (void)hipStreamSynchronize(c->stream);
    if (c->ws) dev_free(c, c->ws, c->ws_bytes);
    if (c->ws2) dev_free(c, c->ws2, c->ws2_bytes);
    (void)hipStreamSynchronize(c->stream);
    if (c->host) (void)hipHostFree(c->host);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

sline_status sline_build(sline_ctx *c, sline_csr H, int32_t s, int32_t dual, uint32_t flags,
                         sline_edges *out) {
    if (!c) return SLINE_EINVAL;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return build_impl(c, H, s, dual, flags, out);
    } catch (const Fail &f) {
        c->pending.valid = false;
        release_pool(c);
        return f.st;
    } catch (const std::bad_alloc &) {
        c->pending.valid = false;
        release_pool(c);
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

sline_status sline_build_noalloc(sline_ctx *c, sline_csr H, int32_t s, int32_t dual,
                                 uint32_t flags, sline_edges *out) {
    if (!c) return SLINE_EINVAL;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return noalloc_impl(c, H, s, dual, flags, out);
    } catch (const Fail &f) {
        c->pending.valid = false;
        return f.st;
    } catch (const std::bad_alloc &) {
        c->pending.valid = false;
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

sline_status sline_build_batch(sline_ctx *c, int32_t n_graphs, const sline_csr *Hs, const int32_t *s,
                               const int32_t *dual, uint32_t flags, sline_edges *outs) {
    if (!c) return SLINE_EINVAL;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return batch_impl(c, n_graphs, Hs, s, dual, flags, outs);
    } catch (const Fail &f) {
        drop_batch_pending(c);
        c->pending.valid = false;
        release_pool(c);
        return f.st;
    } catch (const std::bad_alloc &) {
        drop_batch_pending(c);
        c->pending.valid = false;
        release_pool(c);
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

sline_status sline_batch_plan_create(sline_ctx *c, int32_t n_graphs, const sline_csr *Hs,
                                     const int32_t *s, const int32_t *dual, uint32_t flags,
                                     sline_batch_plan **plan) {
    if (plan) *plan = nullptr;
    if (!c) return SLINE_EINVAL;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return plan_create_impl(c, n_graphs, Hs, s, dual, flags, plan);
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

sline_status sline_batch_plan_run(sline_batch_plan *p, const int32_t *s, sline_edges *outs) {
    if (!p || !p->c) return SLINE_EINVAL;
    sline_ctx *c = p->c;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return plan_run_impl(p, s, outs);
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

sline_status sline_batch_plan_info(const sline_batch_plan *p, int64_t *device_bytes,
                                   int64_t *task_capacity, int64_t *pair_capacity) {
    if (!p) return SLINE_EINVAL;
    int64_t bytes = 0;
    for (const auto &m : p->mem) bytes += (int64_t)m.second;
    if (device_bytes) *device_bytes = bytes;
    if (task_capacity) *task_capacity = p->t_cap;
    if (pair_capacity) *pair_capacity = p->pair_cap;
    return SLINE_OK;
}

void sline_batch_plan_destroy(sline_batch_plan *p) {
    if (!p) return;
    if (p->c) (void)hipSetDevice(p->c->device);
    plan_free(p);
}

sline_status sline_build_spgemm(sline_ctx *c, sline_csr H, int32_t s, int32_t dual, uint32_t flags,
                                sline_edges *out) {
    if (!c) return SLINE_EINVAL;
    c->last_error.clear();
    if (hipSetDevice(c->device) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipSetDevice failed");
        return SLINE_EDEVICE;
    }
    try {
        return spgemm_impl(c, H, s, dual, flags, out);
    } catch (const Fail &f) {
        release_pool(c);
        return f.st;
    } catch (const std::bad_alloc &) {
        set_err(c, "host allocation failed");
        return SLINE_ENOMEM;
    }
}

sline_status sline_edges_free(sline_ctx *c, sline_edges *e) {
    if (!c || !e) return SLINE_EINVAL;
    if (e->capacity == 0) {
        const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(e->n_pairs, 0);
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, e->a, bytes);
        dev_free(c, e->b, bytes);
        dev_free(c, e->w, bytes);
        (void)hipStreamSynchronize(c->stream);
        e->a = e->b = e->w = nullptr;
        e->n_pairs = 0;
    }
    return SLINE_OK;
}

sline_status sline_get_tuning(sline_ctx *c, sline_tuning *t) {
    if (!c || !t) return SLINE_EINVAL;
    t->small_max_wedges = c->tune.small_max_wedges;
    t->task_wedges = c->tune.task_wedges;
    t->group_parts = c->tune.group_parts;
    t->light_len = c->tune.light_len;
    t->small_grid_per_cu = c->tune.small_grid_per_cu;
    t->task_grid_per_cu = c->tune.task_grid_per_cu;
    t->stage_max_bytes = c->tune.stage_max_bytes;
    t->dense_min_wedges = c->tune.dense_min_wedges;
    t->small_slots = c->tune.small_slots;
    t->task_slots = c->tune.task_slots;
    t->tiny_max_wedges = c->tune.tiny_max_wedges;
    return SLINE_OK;
}

sline_status sline_set_tuning(sline_ctx *c, const sline_tuning *t) {
    if (!c || !t) return SLINE_EINVAL;
    auto in = [](int64_t v, int64_t lo, int64_t hi) { return v >= lo && v <= hi; };
    const bool slots_ok = (t->small_slots == 512 || t->small_slots == 1024 ||
                           t->small_slots == 2048) &&
                          (t->task_slots == 4480 || t->task_slots == 8960 ||
                           t->task_slots == 13440 || t->task_slots == 17920);
    if (!slots_ok || !in(t->small_max_wedges, 0, t->small_slots / 2) ||
        !in(t->task_wedges, 64, 1 << 20) ||
        !in(t->group_parts, 1, 1024) || !in(t->light_len, 0, 64) ||
        !in(t->small_grid_per_cu, 1, 64) || !in(t->task_grid_per_cu, 1, 16) ||
        t->stage_max_bytes < 0 || !in(t->dense_min_wedges, 0, 1 << 24) ||
        !in(t->tiny_max_wedges, 0, kTinyMaxCost)) {
        c->last_error = "tuning value out of range";
        return SLINE_EINVAL;
    }
    c->pending.valid = false;
    c->tune.small_max_wedges = t->small_max_wedges;
    c->tune.task_wedges = t->task_wedges;
    c->tune.group_parts = t->group_parts;
    c->tune.light_len = t->light_len;
    c->tune.small_grid_per_cu = t->small_grid_per_cu;
    c->tune.task_grid_per_cu = t->task_grid_per_cu;
    c->tune.stage_max_bytes = t->stage_max_bytes;
    c->tune.dense_min_wedges = t->dense_min_wedges;
    c->tune.small_slots = t->small_slots;
    c->tune.task_slots = t->task_slots;
    c->tune.tiny_max_wedges = t->tiny_max_wedges;
    return SLINE_OK;
}

sline_status sline_last_stats(sline_ctx *c, sline_stats *s) {
    if (!c || !s) return SLINE_EINVAL;
    *s = c->stats;
    return SLINE_OK;
}

const char *sline_status_str(sline_status s) {
    switch (s) {
        case SLINE_OK: return "ok";
        case SLINE_EINVAL: return "invalid argument";
        case SLINE_ENOMEM: return "out of memory";
        case SLINE_ECAPACITY: return "output capacity too small";
        case SLINE_EDEVICE: return "device error";
        case SLINE_EBUSY: return "not ready";
        default: return "unknown status";
    }
}

const char *sline_last_error(sline_ctx *c) { return c ? c->last_error.c_str() : "no context"; }

}  // extern "C"

extern "C" {

sline_status sline_filter(sline_ctx *c, const sline_edges *in, int32_t s, uint32_t flags,
                          sline_edges *out) {
    return guarded(c, [&]() { return filter_impl(c, in, s, flags, out); });
}

sline_status sline_build_sweep(sline_ctx *c, sline_csr H, int32_t n_s, const int32_t *s_list,
                               int32_t dual, uint32_t flags, sline_edges *outs) {
    return guarded(c, [&]() { return sweep_impl(c, H, n_s, s_list, dual, flags, outs); });
}

sline_status sline_squeeze(sline_ctx *c, int32_t n_items, const sline_edges *L, uint32_t flags,
                           sline_graph *G) {
    return guarded(c, [&]() { return squeeze_impl(c, n_items, L, flags, G); });
}

sline_status sline_graph_free(sline_ctx *c, sline_graph *G) {
    if (!c || !G) return SLINE_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, G->old_id, sizeof(int32_t) * (size_t)std::max(G->n_nodes, 1));
    dev_free(c, G->row_ptr, sizeof(int64_t) * ((size_t)G->n_nodes + 1));
    dev_free(c, G->col, sizeof(int32_t) * (size_t)std::max<int64_t>(G->n_arcs, 1));
    dev_free(c, G->w, sizeof(int32_t) * (size_t)std::max<int64_t>(G->n_arcs, 1));
    (void)hipStreamSynchronize(c->stream);
    *G = sline_graph{};
    return SLINE_OK;
}

sline_status sline_components(sline_ctx *c, int32_t n_items, const sline_edges *L, int32_t *comp,
                              int64_t *n_components) {
    return guarded(c, [&]() { return components_impl(c, n_items, L, comp, n_components); });
}

}  // extern "C"
