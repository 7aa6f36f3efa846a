// Batched builds: many hypergraphs, each with its own s and role (primal or
// dual), counted in one pass of the plain pipeline.
//
// The graphs are independent, so their items can share one id space: graph
// g's items take the ids [ibase_g, ibase_g + N_g) and its members the ids
// [mbase_g, mbase_g + M_g).  Two items of different graphs share no member,
// so the combined L_s (each item compared with its own graph's s) is the
// disjoint union of the graphs' L_s, and sorting by (a, b) keeps every
// graph's pairs contiguous.  The kernels here build the combined item CSR
// (checking every caller CSR on the way), give every item its graph's s,
// and hand the combined result back per graph: directly, when the library
// allocates the results (the fill writes each pair into its graph's arrays),
// or by splitting a combined result into caller buffers.
//
// A dual graph's items are its vertices: their member lists are the rows of
// H_g^T, built by transposing XD, the row concatenation of all dual graphs'
// H_g (columns shifted by vdbase_g so the graphs' vertices do not collide).
#include <algorithm>

#include "sline_internal.h"

namespace sl {

namespace {

inline int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
    const int64_t g = (work + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// last g with base[g] <= x, for base ascending with base[0] = 0 <= x
__device__ __forceinline__ int32_t find_graph(const int64_t *base, int32_t G, int64_t x) {
    int32_t lo = 0, hi = G;  // base[lo] <= x < base[hi] (base[G] = total)
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Per graph: nnz (row_ptr[m]) and the row_ptr[0] == 0 check.
__global__ void k_batch_nnz(const BatchGraph *gr, int32_t G, int64_t *nnz, int32_t *err) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const BatchGraph d = gr[g];
    int64_t z = 0;
    if (d.m > 0) {
        if (d.rp[0] != 0) atomicOr(err, kErrRowPtr0);
        z = d.rp[d.m];
    }
    nnz[g] = z;
}

// One wave per row of XD (the dual graphs' rows, in graph order): columns
// shifted by vdbase and the row id of every entry (what the transpose reads);
// range and order checks.
__global__ __launch_bounds__(256) void k_batch_concat(const BatchGraph *gr, const int32_t *dual_ids,
                                                      const int64_t *dbase, int32_t GD, int64_t E,
                                                      int32_t *xcol, int32_t *xrow, int32_t *err) {
    if (*err & kErrPlanShape) return;  // a replayed plan keeps its last lists
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t e = wave; e < E; e += nwaves) {
        const int32_t q = find_graph(dbase, GD, e);
        const BatchGraph d = gr[dual_ids[q]];
        const int32_t loc = (int32_t)(e - dbase[q]);
        const int32_t b = d.rp[loc], en = d.rp[loc + 1];
        // a row outside [0, nnz) is reported and never read (its entries of
        // XD stay zero, so later kernels index safely until the error returns)
        if (b < 0 || en < b || en > d.nnz) {
            if (lane == 0) atomicOr(err, kErrRowPtrOrder);
            continue;
        }
        int32_t bad = 0;
        for (int32_t k = b + lane; k < en; k += kWave) {
            const int32_t v = d.col[k];
            if (v < 0 || v >= d.n) bad |= kErrColRange;
            if (k > b && d.col[k - 1] >= v) bad |= kErrColOrder;
            const int64_t o = d.dzbase + k;
            xcol[o] = (v >= 0 && v < d.n) ? (int32_t)(d.vdbase + v) : 0;
            xrow[o] = (int32_t)e;
        }
        if (bad) atomicOr(err, bad);
    }
}

// One thread per combined item: its row length, its graph's s and the end of
// its graph's items (candidates of an item never lie beyond it).
__global__ void k_batch_len(const BatchGraph *gr, const int64_t *ibase, int32_t G, int64_t NI,
                            const int32_t *ptrT, int32_t *len, int32_t *s_item, int32_t *item_end,
                            int32_t *err) {
    if (*err & kErrPlanShape) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NI;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = find_graph(ibase, G, i);
        const BatchGraph d = gr[g];
        const int32_t loc = (int32_t)(i - ibase[g]);
        int32_t l;
        if (d.dual) {
            const int64_t r = d.vdbase + loc;
            l = ptrT[r + 1] - ptrT[r];
        } else {
            const int32_t b = d.rp[loc], en = d.rp[loc + 1];
            l = en - b;
            if (b < 0 || en < b || en > d.nnz) {
                atomicOr(err, kErrRowPtrOrder);
                l = 0;
            }
            // members: the range is checked per incidence by k_batch_rows,
            // the order within each row on the combined lists (the combined
            // member ids of a primal graph keep its members' order)
        }
        len[i] = l;
        s_item[i] = d.s;
        item_end[i] = (int32_t)ibase[g + 1];
    }
}

// First combined incidence of every graph: zb[g] = ptrC[ibase[g]], g = 0..G.
__global__ void k_batch_zbase(const int64_t *ibase, int32_t G, const int32_t *ptrC, int32_t *zb) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= G) zb[g] = ptrC[ibase[g]];
}

// One thread per combined incidence z (grid-stride).  Graph g's incidences
// are the contiguous range [zb[g], zb[g + 1]) in graph order: a primal
// graph's are its col array (rows checked by k_batch_len), shifted to the
// combined member ids; a dual graph's are its block of XD^T (rows of its
// vertices), whose entries are combined row ids of XD turned into member ids.
__global__ void k_batch_rows(const BatchGraph *gr, const int32_t *zb, int32_t G, int64_t ZT,
                             const int32_t *ptrT, const int32_t *colT, int32_t *memC,
                             int32_t *err) {
    if (*err & kErrPlanShape) return;
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < ZT;
         z += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = G;  // zb[lo] <= z < zb[hi]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if ((int64_t)zb[mid] <= z) lo = mid;
            else hi = mid;
        }
        const BatchGraph d = gr[lo];
        const int64_t k = z - zb[lo];
        if (d.dual) {
            memC[z] = (int32_t)(colT[ptrT[d.vdbase] + k] - d.dbase + d.mbase);
        } else {
            // a graph with bad row bounds (reported by k_batch_len) may map
            // past its col
            const int32_t v = k < d.nnz ? d.col[k] : -1;
            const bool in = v >= 0 && v < d.n;
            if (!in && k < d.nnz) atomicOr(err, kErrColRange);
            memC[z] = in ? (int32_t)(d.mbase + v) : (int32_t)d.mbase;
        }
    }
}

// One thread per graph: first pair of the graph in the combined result
// (items of graph g are [ibase_g, ibase_{g+1}); `a` is sorted).
__global__ void k_batch_bounds(const int64_t *ibase, int32_t G, const int32_t *a, int64_t P,
                               int64_t *off) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > G) return;
    if (g == G) {
        off[G] = P;
        return;
    }
    const int64_t key = ibase[g];
    int64_t lo = 0, hi = P;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    off[g] = lo;
}

// Grid-stride over the combined pairs: each goes to its graph's output with
// the graph's item base taken off both ids.
__global__ void k_batch_split(const int64_t *ibase, const int64_t *off, int32_t G,
                              const int32_t *a, const int32_t *b, const int32_t *w, int64_t P,
                              int32_t *const *oa, int32_t *const *ob, int32_t *const *ow) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = find_graph(off, G, k);
        const int64_t r = k - off[g];
        const int32_t base = (int32_t)ibase[g];
        oa[g][r] = a[k] - base;
        ob[g][r] = b[k] - base;
        if (w && ow[g]) ow[g][r] = w[k];
    }
}

// One thread per graph boundary g = 0..G: the first pair of graph g.
__global__ void k_batch_graph_off(const int32_t *task_item, int32_t T, const int64_t *task_off,
                                  const int64_t *g_ibase, int32_t G, int64_t *g_off,
                                  const int64_t *T_dev) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > G) return;
    if (T_dev) T = (int32_t)min(*T_dev, (int64_t)T);
    const int64_t first = g_ibase[g];
    int32_t lo = 0, hi = T;  // first task with task_item >= first
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int64_t)task_item[mid] < first) lo = mid + 1;
        else hi = mid;
    }
    g_off[g] = task_off[lo];
}

// Replayed plans: the caller's row_ptr must still start at 0 and end at the
// nnz the plan was sized for (every later kernel bounds its reads by it).
__global__ void k_plan_check_shape(const BatchGraph *gr, int32_t G, int32_t *err) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const BatchGraph d = gr[g];
    if (d.m > 0 && (d.rp[0] != 0 || (int64_t)d.rp[d.m] != d.nnz)) atomicOr(err, kErrPlanShape);
}

__global__ void k_plan_guard(const int64_t *value, int64_t cap, int32_t bit, int32_t *err) {
    if (threadIdx.x == 0 && *value > cap) atomicOr(err, bit);
}

}  // namespace

hipError_t launch_batch_graph_off(hipStream_t st, const int32_t *task_item, int32_t n_tasks,
                                  const int64_t *task_off, const int64_t *g_ibase, int32_t G,
                                  int64_t *g_off, const int64_t *n_tasks_dev) {
    if (G <= 0) return hipSuccess;
    k_batch_graph_off<<<grid_for((int64_t)G + 1, 256), 256, 0, st>>>(task_item, n_tasks, task_off,
                                                                     g_ibase, G, g_off, n_tasks_dev);
    return hipGetLastError();
}

hipError_t launch_plan_check_shape(hipStream_t st, const BatchGraph *gr, int32_t G, int32_t *err) {
    if (G <= 0) return hipSuccess;
    k_plan_check_shape<<<grid_for(G, 256), 256, 0, st>>>(gr, G, err);
    return hipGetLastError();
}

hipError_t launch_plan_guard(hipStream_t st, const int64_t *value, int64_t cap, int32_t bit,
                             int32_t *err) {
    k_plan_guard<<<1, kWave, 0, st>>>(value, cap, bit, err);
    return hipGetLastError();
}

hipError_t launch_batch_nnz(hipStream_t st, const BatchGraph *gr, int32_t G, int64_t *nnz,
                            int32_t *err) {
    if (G <= 0) return hipSuccess;
    k_batch_nnz<<<grid_for(G, 256), 256, 0, st>>>(gr, G, nnz, err);
    return hipGetLastError();
}

hipError_t launch_batch_concat(hipStream_t st, const BatchGraph *gr, const int32_t *dual_ids,
                               const int64_t *dbase, int32_t GD, int64_t E, int32_t *xcol,
                               int32_t *xrow, int32_t *err) {
    if (E <= 0) return hipSuccess;
    k_batch_concat<<<grid_for(E * kWave, 256, 65536), 256, 0, st>>>(gr, dual_ids, dbase, GD, E, xcol,
                                                                    xrow, err);
    return hipGetLastError();
}

hipError_t launch_batch_len(hipStream_t st, const BatchGraph *gr, const int64_t *ibase, int32_t G,
                            int64_t NI, const int32_t *ptrT, int32_t *len, int32_t *s_item,
                            int32_t *item_end, int32_t *err) {
    if (NI <= 0) return hipSuccess;
    k_batch_len<<<grid_for(NI, 256, 65536), 256, 0, st>>>(gr, ibase, G, NI, ptrT, len, s_item,
                                                          item_end, err);
    return hipGetLastError();
}

hipError_t launch_batch_rows(hipStream_t st, const BatchGraph *gr, const int64_t *ibase, int32_t G,
                             int64_t ZT, const int32_t *ptrT, const int32_t *colT,
                             const int32_t *ptrC, int32_t *zb, int32_t *memC, int32_t *err) {
    if (G <= 0) return hipSuccess;
    k_batch_zbase<<<grid_for((int64_t)G + 1, 256), 256, 0, st>>>(ibase, G, ptrC, zb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ZT <= 0) return e;
    k_batch_rows<<<grid_for(ZT, 256, 65536), 256, 0, st>>>(gr, zb, G, ZT, ptrT, colT, memC, err);
    return hipGetLastError();
}

hipError_t launch_batch_bounds(hipStream_t st, const int64_t *ibase, int32_t G, const int32_t *a,
                               int64_t P, int64_t *off) {
    k_batch_bounds<<<grid_for((int64_t)G + 1, 256), 256, 0, st>>>(ibase, G, a, P, off);
    return hipGetLastError();
}

hipError_t launch_batch_split(hipStream_t st, const int64_t *ibase, const int64_t *off, int32_t G,
                              const int32_t *a, const int32_t *b, const int32_t *w, int64_t P,
                              int32_t *const *oa, int32_t *const *ob, int32_t *const *ow) {
    if (P <= 0) return hipSuccess;
    k_batch_split<<<grid_for(P, 256, 65536), 256, 0, st>>>(ibase, off, G, a, b, w, P, oa, ob, ow);
    return hipGetLastError();
}

}  // namespace sl
