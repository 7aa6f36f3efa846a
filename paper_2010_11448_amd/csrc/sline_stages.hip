// Stages around the s-line graph for gfx950: the pipeline steps after L_s
// that the paper's Table I times (ID squeezing with the adjacency it makes
// possible, s-connected components), L_s from a weighted L_s' (the s-sweep),
// relabel-by-degree (Sec. IV-F), the per-wedge set intersection of the
// variants without visited skipping (Table III), and the sort of pairs into
// canonical (a, b) order that the last two need.
#include <algorithm>

#include "sline_internal.h"

namespace sl {

namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

inline unsigned grid_for(int64_t work, int per_block, int cap) {
    const int64_t g = (work + per_block - 1) / per_block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ------------------------------------------------------------ filter

// L_s from a weighted L_s' (s' <= s): the pairs with w >= s, in their order
// (Sec. III: L_s keeps the pairs of L_1 with w >= s, with the same w).  A
// tile is four waves of kFtRounds rounds of 64 consecutive pairs; a wave's
// kept pairs go out in round order, so the output keeps the input order.
constexpr int kFtRounds = 16;
constexpr int kFtTile = 4 * kFtRounds * kWave;

__global__ __launch_bounds__(256) void k_wfilter(const int32_t *a, const int32_t *b,
                                                 const int32_t *w, int64_t n, int32_t s,
                                                 int32_t *cnt, const int64_t *off, int32_t *oa,
                                                 int32_t *ob, int32_t *ow) {
    __shared__ int32_t wsum[4];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kFtTile + (int64_t)wid * kFtRounds * kWave;
    int32_t mine = 0;
#pragma unroll
    for (int r = 0; r < kFtRounds; ++r) {
        const int64_t k = base + r * kWave + lane;
        mine += __popcll(__ballot(k < n && w[k] >= s));
    }
    if (lane == 0) wsum[wid] = mine;
    __syncthreads();
    if (!oa) {
        if (threadIdx.x == 0) cnt[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        return;
    }
    int64_t pos = off[blockIdx.x];
    for (int i = 0; i < wid; ++i) pos += wsum[i];
#pragma unroll
    for (int r = 0; r < kFtRounds; ++r) {
        const int64_t k = base + r * kWave + lane;
        const bool keep = k < n && w[k] >= s;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int64_t q = pos + lanes_below(m);
            oa[q] = a[k];
            ob[q] = b[k];
            if (ow) ow[q] = w[k];
        }
        pos += __popcll(m);
    }
}

// ------------------------------------------------- squeeze, adjacency

// flag[x] = 1 for every item x that occurs in a pair.
__global__ void k_mark_present(const int32_t *a, const int32_t *b, int64_t n, int32_t N,
                               int32_t *flag, int32_t *err) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = a[e], y = b[e];
        if (x < 0 || x >= N || y < 0 || y >= N || x >= y) {
            atomicOr(err, kErrColRange);
            continue;
        }
        flag[x] = 1;
        flag[y] = 1;
    }
}

// old_id[newid[x]] = x for the items present.
__global__ void k_old_ids(const int32_t *flag, const int32_t *newid, int32_t N, int32_t *old_id) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x)
        if (flag[x]) old_id[newid[x]] = (int32_t)x;
}

// Starts of the pair runs by first item in a sorted edge list: ptr[x] = the
// first pair with a >= x, for x = 0..N (pairs out of order or range are
// reported by k_mark_present; here they are clamped).
__global__ void k_run_starts(const int32_t *a, int64_t n, int32_t N, int64_t *ptr) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= n;
         p += (int64_t)gridDim.x * blockDim.x) {
        int32_t hi = p < n ? a[p] : N;
        int32_t lo = p > 0 ? a[p - 1] : -1;
        hi = hi < 0 ? 0 : (hi > N ? N : hi);
        lo = lo < -1 ? -1 : (lo > N ? N : lo);
        for (int32_t v = lo + 1; v <= hi; ++v) ptr[v] = p;
    }
}

// Edge list sorted by (a, b)?  Sets kErrColOrder otherwise.
__global__ void k_check_sorted(const int32_t *a, const int32_t *b, int64_t n, int32_t *err) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const bool ok = a[e - 1] < a[e] || (a[e - 1] == a[e] && b[e - 1] < b[e]);
        if (!ok) atomicOr(err, kErrColOrder);
    }
}

// Degree of every item in the symmetric graph: pairs where it is first
// (fwd) plus pairs where it is second (ptrT, the transpose).
__global__ void k_degrees(const int64_t *fwd, const int32_t *ptrT, int32_t N, int32_t *deg) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x)
        deg[x] = (int32_t)(fwd[x + 1] - fwd[x]) + (ptrT[x + 1] - ptrT[x]);
}

__global__ void k_row_ptr(const int32_t *flag, const int32_t *newid, const int64_t *off,
                          int32_t N, int32_t n_nodes, int64_t *row_ptr) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= N;
         x += (int64_t)gridDim.x * blockDim.x) {
        if (x == N) row_ptr[n_nodes] = off[N];
        else if (flag[x]) row_ptr[newid[x]] = off[x];
    }
}

// Row of node x: first the items before it (b = x, from the transpose, items
// ascending), then the items after it (its own pairs, b ascending); both in
// squeezed ids.  One wave per item.
__global__ __launch_bounds__(256) void k_adj_fill(int32_t N, const int32_t *flag,
                                                  const int32_t *newid, const int64_t *off,
                                                  const int32_t *ptrT, const int32_t *colT,
                                                  const int32_t *kT, const int64_t *fwd,
                                                  const int32_t *b, const int32_t *w,
                                                  int32_t *ocol, int32_t *ow) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t x = wave; x < N; x += nwaves) {
        if (!flag[x]) continue;
        const int64_t o = off[x];
        const int32_t q0 = ptrT[x], q1 = ptrT[x + 1];
        for (int32_t q = q0 + lane; q < q1; q += kWave) {
            ocol[o + (q - q0)] = newid[colT[q]];
            if (ow) ow[o + (q - q0)] = w[kT[q]];
        }
        const int64_t ob = o + (q1 - q0);
        const int64_t e0 = fwd[x], e1 = fwd[x + 1];
        for (int64_t e = e0 + lane; e < e1; e += kWave) {
            ocol[ob + (e - e0)] = newid[b[e]];
            if (ow) ow[ob + (e - e0)] = w[e];
        }
    }
}

// ----------------------------------------------------------- components

__device__ __forceinline__ int32_t ld_rel(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x in the union-find forest p: links only ever point to smaller
// ids, so the walk ends; every node passed is pointed at its grandparent
// (path halving), which keeps the trees shallow.
__device__ __forceinline__ int32_t uf_root(int32_t *p, int32_t x) {
    for (;;) {
        const int32_t px = ld_rel(p + x);
        if (px == x) return x;
        const int32_t gx = ld_rel(p + px);
        if (gx == px) return px;
        st_rel(p + x, gx);
        x = gx;
    }
}

__global__ void k_iota(int32_t *p, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        p[x] = (int32_t)x;
}

// Union of the two ends of every pair: the larger root is linked under the
// smaller with a compare-and-swap that succeeds only while it is still a
// root, so a component's final root is its smallest item.
__global__ void k_cc_hook(const int32_t *a, const int32_t *b, int64_t n, int32_t *p) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t ra = uf_root(p, a[e]), rb = uf_root(p, b[e]);
        while (ra != rb) {
            const int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
            const int32_t old = atomicCAS(p + hi, hi, lo);
            if (old == hi) break;
            ra = uf_root(p, hi);
            rb = uf_root(p, lo);
        }
    }
}

__global__ void k_cc_flatten(int32_t *p, int32_t N) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x)
        st_rel(p + x, uf_root(p, (int32_t)x));
}

// Roots that occur in a pair: one per component of the squeezed graph.
__global__ __launch_bounds__(256) void k_cc_count(const int32_t *comp, const int32_t *flag,
                                                  int32_t N, unsigned long long *count) {
    __shared__ int32_t sh[4];
    int32_t mine = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x)
        mine += flag[x] && comp[x] == x;
    for (int d = 32; d >= 1; d >>= 1) mine += __shfl_xor(mine, d, kWave);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t t = sh[0] + sh[1] + sh[2] + sh[3];
        if (t) atomicAdd(count, (unsigned long long)t);
    }
}

// ------------------------------------------------------------ gathers

__global__ void k_gather(const int32_t *src, const int32_t *idx, int64_t n, int32_t *dst) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = src[idx[q]];
}

// (perm[a], perm[b]) with the smaller first.
__global__ void k_map_pairs(const int32_t *a, const int32_t *b, int64_t n, const int32_t *perm,
                            int32_t *oa, int32_t *ob) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = perm[a[q]], y = perm[b[q]];
        oa[q] = x < y ? x : y;
        ob[q] = x < y ? y : x;
    }
}

// ------------------------------------------------------------- relabel

// Size of each item of a side: the row lengths of its item lists.
__global__ void k_sizes(const int32_t *ptr, int32_t N, int32_t *size, int32_t *max_size) {
    int32_t m = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x) {
        size[x] = ptr[x + 1] - ptr[x];
        m = size[x] > m ? size[x] : m;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const int32_t o = __shfl_xor(m, d, kWave);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && m) atomicMax(max_size, m);
}

// Sort key of an item: its size (ascending order) or max - size (descending).
__global__ void k_size_keys(const int32_t *size, int32_t N, const int32_t *max_size,
                            int32_t descending, int32_t *key) {
    const int32_t mx = *max_size;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x)
        key[x] = descending ? mx - size[x] : size[x];
}

__global__ void k_invert(const int32_t *perm, int32_t N, int32_t *inv) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x)
        inv[perm[k]] = (int32_t)k;
}

// len[k] = size of old row perm[k].
__global__ void k_perm_lengths(const int32_t *rp, const int32_t *perm, int32_t N, int32_t *len) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x)
        len[k] = rp[perm[k] + 1] - rp[perm[k]];
}

// Row k of the relabeled CSR is old row perm[k]; one wave per row.
__global__ __launch_bounds__(256) void k_perm_rows(const int32_t *rp, const int32_t *col,
                                                   const int32_t *perm, const int32_t *nrp,
                                                   int32_t N, int32_t *ncol) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t k = wave; k < N; k += nwaves) {
        const int32_t s0 = rp[perm[k]], len = rp[perm[k] + 1] - s0, d0 = nrp[k];
        for (int32_t i = lane; i < len; i += kWave) ncol[d0 + i] = col[s0 + i];
    }
}

// Row id of every incidence of a CSR (one wave per row).
__global__ __launch_bounds__(256) void k_row_ids(const int32_t *rp, int32_t m, int32_t *rowid) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = wave; r < m; r += nwaves)
        for (int32_t k = rp[r] + lane; k < rp[r + 1]; k += kWave) rowid[k] = (int32_t)r;
}

// ------------------------------------------------ no visited skipping

// The variants of Table III without visited skipping make one set
// intersection per wedge (a, v, b), b > a: |S_a & S_b| by a two-pointer merge
// of the sorted member lists, stopping at s common members when short-
// circuiting.  A pair accepted through several shared members enters L_s once
// (it is a set): it is emitted by its first common member, which the merge
// meets first.  One workgroup per item; count mode adds the item's accepted
// pairs to cnt[a], write mode appends them (in any order) from off[a].
__device__ __forceinline__ void merge_first(const int32_t *x, int32_t nx, const int32_t *y,
                                            int32_t ny, int32_t s, int32_t shortcut, int32_t &c,
                                            int32_t &first) {
    int32_t i = 0, j = 0;
    c = 0;
    first = -1;
    while (i < nx && j < ny) {
        const int32_t u = x[i], v = y[j];
        if (u < v) {
            ++i;
        } else if (v < u) {
            ++j;
        } else {
            if (c == 0) first = u;
            ++c;
            ++i;
            ++j;
            if (shortcut && c >= s) return;
        }
    }
}

constexpr int kNvThreads = 256;

__global__ __launch_bounds__(kNvThreads) void k_wedge_intersect(
    const int32_t *ptrI, const int32_t *memI, const int32_t *ptrS, const int32_t *itmS,
    const int32_t *start, int32_t N, int32_t s, int32_t prune, int32_t shortcut, int32_t *cnt,
    const int64_t *off, int32_t *oa, int32_t *ob, int32_t *ow, unsigned long long *inters) {
    __shared__ int32_t fill;
    __shared__ unsigned long long made;
    if (threadIdx.x == 0) made = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (int32_t a = blockIdx.x; a < N; a += gridDim.x) {
        const int32_t k0 = ptrI[a], k1 = ptrI[a + 1];
        if (k1 == k0 || (prune && k1 - k0 < s)) continue;
        if (threadIdx.x == 0) fill = 0;
        __syncthreads();
        const int32_t *Sa = memI + k0;
        // wedges of a: for member v (incidence k), the kept items after a in
        // N(v), from the back-pointer start[k] to the list end
        for (int32_t k = k0; k < k1; ++k) {
            const int32_t v = memI[k];
            const int32_t q0 = start[k] & kStartMask, q1 = ptrS[v + 1];
            for (int32_t q = q0 + (int32_t)threadIdx.x; q < q1; q += kNvThreads) {
                const int32_t bi = itmS[q];
                const int32_t *Sb = memI + ptrI[bi];
                const int32_t nb = ptrI[bi + 1] - ptrI[bi];
                int32_t c, first;
                merge_first(Sa, k1 - k0, Sb, nb, s, shortcut, c, first);
                ++mine;
                if (c >= s && first == v) {
                    int32_t wv = c;
                    if (shortcut) merge_first(Sa, k1 - k0, Sb, nb, s, 0, wv, first);
                    const int32_t slot = atomicAdd(&fill, 1);
                    if (oa) {
                        const int64_t o = off[a] + slot;
                        oa[o] = a;
                        ob[o] = bi;
                        if (ow) ow[o] = wv;
                    }
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0 && !oa) cnt[a] = fill;
        __syncthreads();
    }
    if (inters) {
        atomicAdd(&made, mine);
        __syncthreads();
        if (threadIdx.x == 0 && made) atomicAdd(inters, made);
    }
}

}  // namespace

// ------------------------------------------------------------ launchers

int64_t wfilter_tiles(int64_t n) { return (n + kFtTile - 1) / kFtTile; }

hipError_t launch_wfilter(hipStream_t st, const int32_t *a, const int32_t *b, const int32_t *w,
                          int64_t n, int32_t s, int32_t *cnt, const int64_t *off, int32_t *oa,
                          int32_t *ob, int32_t *ow) {
    if (n <= 0) return hipSuccess;
    k_wfilter<<<(unsigned)wfilter_tiles(n), 256, 0, st>>>(a, b, w, n, s, cnt, off, oa, ob, ow);
    return hipGetLastError();
}

hipError_t launch_mark_present(hipStream_t st, const int32_t *a, const int32_t *b, int64_t n,
                               int32_t N, int32_t *flag, int32_t *err) {
    if (n <= 0) return hipSuccess;
    k_mark_present<<<grid_for(n, 256, 65536), 256, 0, st>>>(a, b, n, N, flag, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n < 2) return e;
    k_check_sorted<<<grid_for(n, 256, 65536), 256, 0, st>>>(a, b, n, err);
    return hipGetLastError();
}

hipError_t launch_old_ids(hipStream_t st, const int32_t *flag, const int32_t *newid, int32_t N,
                          int32_t *old_id) {
    if (N <= 0) return hipSuccess;
    k_old_ids<<<grid_for(N, 256, 65536), 256, 0, st>>>(flag, newid, N, old_id);
    return hipGetLastError();
}

hipError_t launch_run_starts(hipStream_t st, const int32_t *a, int64_t n, int32_t N, int64_t *ptr) {
    k_run_starts<<<grid_for(n + 1, 256, 65536), 256, 0, st>>>(a, n, N, ptr);
    return hipGetLastError();
}

hipError_t launch_degrees(hipStream_t st, const int64_t *fwd, const int32_t *ptrT, int32_t N,
                          int32_t *deg) {
    if (N <= 0) return hipSuccess;
    k_degrees<<<grid_for(N, 256, 65536), 256, 0, st>>>(fwd, ptrT, N, deg);
    return hipGetLastError();
}

hipError_t launch_row_ptr(hipStream_t st, const int32_t *flag, const int32_t *newid,
                          const int64_t *off, int32_t N, int32_t n_nodes, int64_t *row_ptr) {
    k_row_ptr<<<grid_for((int64_t)N + 1, 256, 65536), 256, 0, st>>>(flag, newid, off, N, n_nodes,
                                                                    row_ptr);
    return hipGetLastError();
}

hipError_t launch_adj_fill(hipStream_t st, int32_t N, const int32_t *flag, const int32_t *newid,
                           const int64_t *off, const int32_t *ptrT, const int32_t *colT,
                           const int32_t *kT, const int64_t *fwd, const int32_t *b,
                           const int32_t *w, int32_t *ocol, int32_t *ow) {
    if (N <= 0) return hipSuccess;
    k_adj_fill<<<grid_for((int64_t)N * kWave, 256, 16384), 256, 0, st>>>(
        N, flag, newid, off, ptrT, colT, kT, fwd, b, w, ocol, ow);
    return hipGetLastError();
}

hipError_t launch_iota(hipStream_t st, int32_t *p, int64_t n) {
    if (n <= 0) return hipSuccess;
    k_iota<<<grid_for(n, 256, 65536), 256, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_components(hipStream_t st, const int32_t *a, const int32_t *b, int64_t n,
                             int32_t N, int32_t *comp) {
    if (N <= 0) return hipSuccess;
    hipError_t e = launch_iota(st, comp, N);
    if (e != hipSuccess) return e;
    if (n > 0) {
        k_cc_hook<<<grid_for(n, 256, 65536), 256, 0, st>>>(a, b, n, comp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_cc_flatten<<<grid_for(N, 256, 65536), 256, 0, st>>>(comp, N);
    return hipGetLastError();
}

hipError_t launch_cc_count(hipStream_t st, const int32_t *comp, const int32_t *flag, int32_t N,
                           unsigned long long *count) {
    if (N <= 0) return hipSuccess;
    k_cc_count<<<grid_for(N, 256, 4096), 256, 0, st>>>(comp, flag, N, count);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t st, const int32_t *src, const int32_t *idx, int64_t n,
                         int32_t *dst) {
    if (n <= 0) return hipSuccess;
    k_gather<<<grid_for(n, 256, 65536), 256, 0, st>>>(src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_map_pairs(hipStream_t st, const int32_t *a, const int32_t *b, int64_t n,
                            const int32_t *perm, int32_t *oa, int32_t *ob) {
    if (n <= 0) return hipSuccess;
    k_map_pairs<<<grid_for(n, 256, 65536), 256, 0, st>>>(a, b, n, perm, oa, ob);
    return hipGetLastError();
}

hipError_t launch_sizes(hipStream_t st, const int32_t *ptr, int32_t N, int32_t *size,
                        int32_t *max_size) {
    if (N <= 0) return hipSuccess;
    k_sizes<<<grid_for(N, 256, 65536), 256, 0, st>>>(ptr, N, size, max_size);
    return hipGetLastError();
}

hipError_t launch_size_keys(hipStream_t st, const int32_t *size, int32_t N, const int32_t *max_size,
                            int32_t descending, int32_t *key) {
    if (N <= 0) return hipSuccess;
    k_size_keys<<<grid_for(N, 256, 65536), 256, 0, st>>>(size, N, max_size, descending, key);
    return hipGetLastError();
}

hipError_t launch_invert(hipStream_t st, const int32_t *perm, int32_t N, int32_t *inv) {
    if (N <= 0) return hipSuccess;
    k_invert<<<grid_for(N, 256, 65536), 256, 0, st>>>(perm, N, inv);
    return hipGetLastError();
}

hipError_t launch_perm_rows(hipStream_t st, const int32_t *rp, const int32_t *col,
                            const int32_t *perm, int32_t N, int32_t *len, int32_t *nrp,
                            int32_t *part32, int32_t *ncol) {
    if (N <= 0) return launch_fill_i32(st, nrp, 1, 0);
    k_perm_lengths<<<grid_for(N, 256, 65536), 256, 0, st>>>(rp, perm, N, len);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_i32(st, len, N, nrp, part32);
    if (e != hipSuccess) return e;
    k_perm_rows<<<grid_for((int64_t)N * kWave, 256, 16384), 256, 0, st>>>(rp, col, perm, nrp, N,
                                                                          ncol);
    return hipGetLastError();
}

hipError_t launch_row_ids(hipStream_t st, const int32_t *rp, int32_t m, int32_t *rowid) {
    if (m <= 0) return hipSuccess;
    k_row_ids<<<grid_for((int64_t)m * kWave, 256, 16384), 256, 0, st>>>(rp, m, rowid);
    return hipGetLastError();
}

hipError_t launch_wedge_intersect(hipStream_t st, const int32_t *ptrI, const int32_t *memI,
                                  const int32_t *ptrS, const int32_t *itmS, const int32_t *start,
                                  int32_t N, int32_t s, int32_t prune, int32_t shortcut,
                                  int32_t *cnt, const int64_t *off, int32_t *oa, int32_t *ob,
                                  int32_t *ow, unsigned long long *inters, int32_t n_cu) {
    if (N <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::max(1, std::min(N, n_cu * 8));
    k_wedge_intersect<<<g, kNvThreads, 0, st>>>(ptrI, memI, ptrS, itmS, start, N, s, prune,
                                                shortcut, cnt, off, oa, ob, ow, inters);
    return hipGetLastError();
}

}  // namespace sl
