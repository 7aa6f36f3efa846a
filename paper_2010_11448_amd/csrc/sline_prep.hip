// Preparation kernels of libsline for gfx950: CSR checks, degree histogram,
// device-wide exclusive scans, the transpose (atomic scatter followed by a
// per-row sort), the s-filtered membership lists, the exact per-item wedge
// count W_a and the degree buckets.
//
// The transpose turns the hyperedge -> vertex incidence lists into vertex ->
// hyperedge lists (the other side of the bipartite representation, Sec. III);
// with both adjacencies the counting kernels walk, for an item a, only the
// items that share a member with it (Sec. IV-B).  Item sizes |S_a| drive the
// degree-based pruning of Sec. IV-C.
#include "sline_internal.h"

namespace sl {

namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan across a 256-thread block; returns the exclusive prefix of
// `v` and writes the block total to `total`.
template <typename T>
__device__ T block_excl_scan(T v, T *sh /* 4 + 1 */, T &total) {
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    T inc = wave_incl_scan(v);
    if (lane == kWave - 1) sh[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            T t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[kScanThreads / kWave] = run;
    }
    __syncthreads();
    T ex = sh[wid] + inc - v;
    total = sh[kScanThreads / kWave];
    __syncthreads();
    return ex;
}

// first index p in [lo, hi) with arr[p] > key (arr ascending), hi if none
__device__ __forceinline__ int32_t upper_bound(const int32_t *arr, int32_t lo, int32_t hi,
                                               int32_t key) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if (arr[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

inline int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ------------------------------------------------------------- checks

__global__ void k_check_rowptr(const int32_t *rp, int32_t m, int32_t *err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && rp[0] != 0) atomicOr(err, kErrRowPtr0);
    if (i < m && rp[i] > rp[i + 1]) atomicOr(err, kErrRowPtrOrder);
}

// One wave per row (grid-stride): the row id of every incidence, member range
// checks and, when asked, the strictly-increasing check of each row.
__global__ __launch_bounds__(256) void k_rows(const int32_t *rp, const int32_t *col, int32_t m,
                                              int32_t n, int64_t nnz, int check_order,
                                              int32_t *rowid, int32_t *err) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    int32_t bad = 0;
    for (int64_t i = wave; i < m; i += nwaves) {
        int64_t b = rp[i], e = rp[i + 1];
        if (b < 0) b = 0;
        if (e > nnz) e = nnz;
        for (int64_t k = b + lane; k < e; k += kWave) {
            int32_t v = col[k];
            rowid[k] = (int32_t)i;
            if (v < 0 || v >= n) bad |= kErrColRange;
            if (check_order && k + 1 < e && col[k + 1] <= v) bad |= kErrColOrder;
        }
    }
    if (bad) atomicOr(err, bad);
}

__global__ void k_degree(const int32_t *col, int64_t nnz, int32_t n, int32_t *deg) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = col[k];
        if (v >= 0 && v < n) atomicAdd(&deg[v], 1);
    }
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_copy(int32_t *dst, const int32_t *src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// --------------------------------------------------------------- scan
// Three phases: per-tile sums, one-block scan of the tile sums, per-tile
// scan plus tile offset.  out has n + 1 entries; out[n] is the total.

template <typename TI, typename TA>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const TI *in, int64_t n,
                                                              TA *partial) {
    __shared__ TA sh[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TA s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) s += (TA)in[base + q];
    TA tot;
    block_excl_scan<TA>(s, sh, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename TA>
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(TA *partial, int64_t nb) {
    __shared__ TA sh[kScanThreads / kWave + 1];
    TA carry = 0;
    for (int64_t c = 0; c < nb; c += kScanTile) {
        const int64_t base = c + (int64_t)threadIdx.x * kScanItems;
        TA v[kScanItems];
        TA s = 0;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            v[q] = (base + q < nb) ? partial[base + q] : (TA)0;
            s += v[q];
        }
        TA tot;
        TA ex = block_excl_scan<TA>(s, sh, tot);
        TA run = carry + ex;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            if (base + q < nb) partial[base + q] = run;
            run += v[q];
        }
        carry += tot;
    }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const TI *in, int64_t n,
                                                            const TO *partial, TO *out) {
    __shared__ TO sh[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TO v[kScanItems];
    TO s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (base + q < n) ? (TO)in[base + q] : (TO)0;
        s += v[q];
    }
    TO tot;
    TO ex = block_excl_scan<TO>(s, sh, tot);
    TO run = partial[blockIdx.x] + ex;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = partial[blockIdx.x] + tot;
}

template <typename TO>
__global__ void k_zero_total(TO *out) { out[0] = 0; }

// ---------------------------------------------------------- transpose

__global__ void k_scatter(const int32_t *col, const int32_t *rowid, int64_t nnz, int32_t n,
                          const int32_t *ptrT, int32_t *fill, int32_t *colT) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = col[k];
        if (v < 0 || v >= n) continue;
        int32_t p = ptrT[v] + atomicAdd(&fill[v], 1);
        colT[p] = (int32_t)k;  // incidence index: within a row it orders like the row id
    }
}

// After the per-row sort of incidence indices: colT[p] becomes the row id of
// incidence kT[p] = colT[p], and posT[k] the transposed position of incidence
// k (kT / posT may be null).
__global__ void k_transpose_fix(int64_t nnz, const int32_t *rowid, int32_t *colT, int32_t *kT,
                                int32_t *posT) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = colT[p];
        if (kT) kT[p] = k;
        if (posT) posT[k] = (int32_t)p;
        colT[p] = rowid[k];
    }
}

// start[k] = map[k] + 1 for every item incidence k (lists not filtered: the
// first item after a in N(v) follows a's own position in the list).
__global__ void k_start_from_map(int64_t nnz, const int32_t *map, int32_t *start) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        start[k] = map[k] + 1;
}

__global__ void k_segsort_classify(const int32_t *ptr, int32_t n, int32_t *mid_list,
                                   int32_t *big_list, int32_t *counts) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t d = ptr[v + 1] - ptr[v];
        if (d > kSegSortSmall && d <= kSegSortLds) mid_list[atomicAdd(&counts[0], 1)] = (int32_t)v;
        else if (d > kSegSortLds) {
            big_list[atomicAdd(&counts[1], 1)] = (int32_t)v;
            atomicMax(&counts[2], d);
        }
    }
}

// Rows of up to kSegSortSmall entries: one thread, insertion sort in place.
__global__ void k_segsort_small(const int32_t *ptr, int32_t n, int32_t *val) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = ptr[v], d = ptr[v + 1] - b;
        if (d < 2 || d > kSegSortSmall) continue;
        int32_t *x = val + b;
        for (int32_t i = 1; i < d; ++i) {
            int32_t key = x[i];
            int32_t j = i - 1;
            while (j >= 0 && x[j] > key) {
                x[j + 1] = x[j];
                --j;
            }
            x[j + 1] = key;
        }
    }
}

// Rows of kSegSortSmall < d <= kSegSortLds entries: one workgroup, bitonic
// sort in LDS padded to a power of two.
__global__ __launch_bounds__(256) void k_segsort_mid(const int32_t *ptr, const int32_t *mid_list,
                                                     const int32_t *counts, int32_t *val) {
    __shared__ int32_t buf[kSegSortLds];
    const int32_t nmid = counts[0];
    for (int32_t r = blockIdx.x; r < nmid; r += gridDim.x) {
        const int32_t v = mid_list[r];
        const int32_t b = ptr[v], d = ptr[v + 1] - b;
        int32_t n2 = 1;
        while (n2 < d) n2 <<= 1;
        for (int32_t i = threadIdx.x; i < n2; i += blockDim.x)
            buf[i] = (i < d) ? val[b + i] : INT32_MAX;
        __syncthreads();
        for (int32_t k = 2; k <= n2; k <<= 1) {
            for (int32_t j = k >> 1; j > 0; j >>= 1) {
                for (int32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                    int32_t l = i ^ j;
                    if (l > i) {
                        int32_t x = buf[i], y = buf[l];
                        bool up = (i & k) == 0;
                        if ((x > y) == up) {
                            buf[i] = y;
                            buf[l] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int32_t i = threadIdx.x; i < d; i += blockDim.x) val[b + i] = buf[i];
        __syncthreads();
    }
}

__global__ void k_big_load(const int32_t *src, int32_t len, int32_t n2, int32_t *tmp) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x)
        tmp[i] = (i < len) ? src[i] : INT32_MAX;
}

__global__ void k_bitonic_step(int32_t *tmp, int32_t n2, int32_t k, int32_t j) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t l = i ^ j;
        if (l > i) {
            int32_t x = tmp[i], y = tmp[l];
            bool up = (i & k) == 0;
            if ((x > y) == up) {
                tmp[i] = y;
                tmp[l] = x;
            }
        }
    }
}

// -------------------------------------------------------- s filtering

// The s filter as a stream compaction: the filtered lists N_s(v), one after
// the other, are the kept entries of the member lists in their order, so the
// position of a kept entry is the number of kept entries before it.
// keep[p] = 1 if entry p of the member lists is an item with |S| >= s
// (s_item[it] for item it when given).
__global__ void k_filter_flags(const int32_t *itmM, int64_t nnz, const int32_t *ptrI, int32_t s,
                               const int32_t *s_item, int32_t *keep) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t it = itmM[p];
        keep[p] = (ptrI[it + 1] - ptrI[it]) >= (s_item ? s_item[it] : s) ? 1 : 0;
    }
}

// After the exclusive scan of the flags (pos[p], pos[nnz] = kept total): kept
// entry p goes to itmS[pos[p]], and the item's own entry sets its
// back-pointer start[inv[p]] to the position after it; ptrS[v] = pos[ptrM[v]].
__global__ void k_filter_scatter(const int32_t *itmM, int64_t nnz, const int32_t *pos,
                                 const int32_t *ptrM, int32_t M, int32_t *ptrS, int32_t *itmS,
                                 const int32_t *inv, int32_t *start) {
    const int64_t n = nnz > (int64_t)M + 1 ? nnz : (int64_t)M + 1;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (p < nnz) {
            const int32_t q = pos[p];
            if (pos[p + 1] != q) {
                itmS[q] = itmM[p];
                if (start) start[inv[p]] = q + 1;
            }
        }
        if (p <= M) ptrS[p] = pos[ptrM[p]];
    }
}

// One wave per item (grid-stride): W_a = sum over members v of the number of
// kept items b > a in N_s(v); 0 for items with |S_a| < s.  For every member
// incidence k of a kept item, start[k] = index in itmS of the first item > a
// in N_s(v) (the back-pointer where a's walk over v begins).
__global__ __launch_bounds__(256) void k_cost(const int32_t *ptrI, const int32_t *memI,
                                              int32_t N, int32_t s, const int32_t *s_item,
                                              const int32_t *ptrS, const int32_t *itmS,
                                              int64_t *cost, int32_t *start, int64_t *totals,
                                              int32_t full, int32_t have_start) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    int64_t kept = 0, kept_nnz = 0, wedges = 0;
    for (int64_t a = wave; a < N; a += nwaves) {
        const int32_t b = ptrI[a], e = ptrI[a + 1];
        if (e - b < (s_item ? s_item[a] : s)) {
            if (lane == 0) cost[a] = 0;
            continue;
        }
        int64_t c = 0;
        for (int32_t k = b + lane; k < e; k += kWave) {
            const int32_t v = memI[k];
            const int32_t lo = ptrS[v], hi = ptrS[v + 1];
            int32_t st;
            if (have_start) {
                st = start[k];
            } else {
                st = full ? lo : upper_bound(itmS, lo, hi, (int32_t)a);
                start[k] = st;
            }
            c += hi - st;
        }
        c = wave_sum(c);
        if (lane == 0) cost[a] = c;
        kept += 1;
        kept_nnz += e - b;
        wedges += c;
    }
    // one atomic per counter and block (same-address atomics serialize)
    __shared__ int64_t red[3][256 / kWave];
    const int wid = threadIdx.x / kWave;
    if (lane == 0) {
        red[0][wid] = kept;
        red[1][wid] = kept_nnz;
        red[2][wid] = wedges;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int64_t t = 0;
        for (int w = 0; w < 256 / kWave; ++w) t += red[threadIdx.x][w];
        if (t) atomicAdd((unsigned long long *)&totals[threadIdx.x], (unsigned long long)t);
    }
}

// One wave per kept item: flag as lookup-only the min(s - 1, kMaxLookup)
// members with the most candidates after a (ties to the lower incidence), by
// setting the sign bit of start[k].  At least one member stays unflagged, as
// |S_a| >= s for a kept item.  The item's planning cost becomes the wedges of
// its inserting members (they fill the table), but at least a third of W_a
// (every wedge is still read).
__global__ __launch_bounds__(256) void k_mark_lookup(const int32_t *ptrI, const int32_t *memI,
                                                     int32_t N, int32_t s_all,
                                                     const int32_t *s_item, const int32_t *ptrS,
                                                     int32_t *start, int64_t *cost) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t a = wave; a < N; a += nwaves) {
        const int32_t b = ptrI[a], e = ptrI[a + 1];
        const int32_t s = s_item ? s_item[a] : s_all;
        if (e - b < s) continue;
        const int32_t rounds = min(min(s - 1, kMaxLookup), e - b - 1);
        int64_t flagged = 0;
        for (int32_t r = 0; r < rounds; ++r) {
            // best unflagged member: most candidates, then lowest k
            uint64_t best = 0;
            for (int32_t k = b + lane; k < e; k += kWave) {
                const int32_t st = start[k];
                if (st < 0) continue;
                const int32_t c = ptrS[memI[k] + 1] - st;
                const uint64_t key = ((uint64_t)(uint32_t)c << 32) | (uint32_t)(INT32_MAX - k);
                best = key > best ? key : best;
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const uint64_t o = __shfl_xor(best, d, kWave);
                best = o > best ? o : best;
            }
            if ((best >> 32) == 0) break;  // no member with candidates left
            const int32_t k = INT32_MAX - (int32_t)(uint32_t)best;
            if (lane == 0) start[k] |= (int32_t)0x80000000u;
            flagged += (int64_t)(best >> 32);
        }
        if (lane == 0 && flagged) {
            const int64_t w = cost[a];
            cost[a] = max(w - flagged, (w + 2) / 3);
        }
    }
}

// Product filter, one block per tile of kFilterTile entries (256 threads x
// 16): pass 1 counts the kept entries of the tile, pass 2 writes them at
// off[tile] in their original order.
__global__ __launch_bounds__(256) void k_product_filter(const int32_t *a, const int32_t *b,
                                                        const int32_t *w, int64_t n, int32_t s,
                                                        int32_t *cnt, const int64_t *off,
                                                        int32_t *oa, int32_t *ob, int32_t *ow) {
    __shared__ int32_t sh[kScanThreads / kWave + 1];
    constexpr int PER = kFilterTile / 256;
    const int64_t t0 = (int64_t)blockIdx.x * kFilterTile;
    int32_t keep[PER];
    int32_t mine = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t k = t0 + (int64_t)threadIdx.x * PER + i;
        keep[i] = k < n && b[k] > a[k] && w[k] >= s;
        mine += keep[i];
    }
    int32_t total;
    const int32_t ex = block_excl_scan<int32_t>(mine, sh, total);
    if (!oa) {
        if (threadIdx.x == 0) cnt[blockIdx.x] = total;
        return;
    }
    int64_t o = off[blockIdx.x] + ex;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        if (keep[i]) {
            const int64_t k = t0 + (int64_t)threadIdx.x * PER + i;
            oa[o] = a[k];
            ob[o] = b[k];
            if (ow) ow[o] = w[k];
            ++o;
        }
    }
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_product_filter(hipStream_t st, const int32_t *a, const int32_t *b, const int32_t *w,
                                 int64_t n, int32_t s, int32_t *cnt, const int64_t *off,
                                 int32_t *out_a, int32_t *out_b, int32_t *out_w) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + kFilterTile - 1) / kFilterTile;
    k_product_filter<<<(unsigned)tiles, 256, 0, st>>>(a, b, w, n, s, cnt, off, out_a, out_b, out_w);
    return hipGetLastError();
}

hipError_t launch_check_rowptr(hipStream_t st, const int32_t *rp, int32_t m, int32_t *err) {
    k_check_rowptr<<<grid_for((int64_t)m + 1, 256), 256, 0, st>>>(rp, m, err);
    return hipGetLastError();
}

hipError_t launch_rows(hipStream_t st, const int32_t *rp, const int32_t *col, int32_t m,
                       int32_t n, int64_t nnz, int check_order, int32_t *rowid, int32_t *err) {
    if (m <= 0) return hipSuccess;
    k_rows<<<grid_for((int64_t)m * kWave, 256, 65536), 256, 0, st>>>(rp, col, m, n, nnz,
                                                                    check_order, rowid, err);
    return hipGetLastError();
}

hipError_t launch_degree(hipStream_t st, const int32_t *col, int64_t nnz, int32_t n,
                         int32_t *deg) {
    if (nnz <= 0) return hipSuccess;
    k_degree<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(col, nnz, n, deg);
    return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t st, int32_t *p, int64_t n, int32_t v) {
    if (n <= 0) return hipSuccess;
    k_fill<int32_t><<<grid_for(n, 256, 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i64(hipStream_t st, int64_t *p, int64_t n, int64_t v) {
    if (n <= 0) return hipSuccess;
    k_fill<int64_t><<<grid_for(n, 256, 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy_i32(hipStream_t st, int32_t *dst, const int32_t *src, int64_t n) {
    if (n <= 0) return hipSuccess;
    k_copy<<<grid_for(n, 256, 65536), 256, 0, st>>>(dst, src, n);
    return hipGetLastError();
}

int64_t scan_partials(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename TI, typename TO>
static hipError_t scan_impl(hipStream_t st, const TI *in, int64_t n, TO *out, TO *partial) {
    if (n <= 0) {
        k_zero_total<TO><<<1, 1, 0, st>>>(out);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    k_scan_reduce<TI, TO><<<(unsigned)nb, kScanThreads, 0, st>>>(in, n, partial);
    k_scan_partials<TO><<<1, kScanThreads, 0, st>>>(partial, nb);
    k_scan_down<TI, TO><<<(unsigned)nb, kScanThreads, 0, st>>>(in, n, partial, out);
    return hipGetLastError();
}

hipError_t launch_scan_i32(hipStream_t st, const int32_t *in, int64_t n, int32_t *out,
                           int32_t *partial) {
    return scan_impl<int32_t, int32_t>(st, in, n, out, partial);
}

hipError_t launch_scan_i32_to_i64(hipStream_t st, const int32_t *in, int64_t n, int64_t *out,
                                  int64_t *partial) {
    return scan_impl<int32_t, int64_t>(st, in, n, out, partial);
}

hipError_t launch_scatter(hipStream_t st, const int32_t *col, const int32_t *rowid, int64_t nnz,
                          int32_t n, const int32_t *ptrT, int32_t *fill, int32_t *colT) {
    if (nnz <= 0) return hipSuccess;
    k_scatter<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(col, rowid, nnz, n, ptrT, fill, colT);
    return hipGetLastError();
}

hipError_t launch_transpose_fix(hipStream_t st, int64_t nnz, const int32_t *rowid, int32_t *colT,
                                int32_t *kT, int32_t *posT) {
    if (nnz <= 0) return hipSuccess;
    k_transpose_fix<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(nnz, rowid, colT, kT, posT);
    return hipGetLastError();
}

hipError_t launch_start_from_map(hipStream_t st, int64_t nnz, const int32_t *map, int32_t *start) {
    if (nnz <= 0) return hipSuccess;
    k_start_from_map<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(nnz, map, start);
    return hipGetLastError();
}

hipError_t launch_segsort_classify(hipStream_t st, const int32_t *ptr, int32_t n,
                                   int32_t *mid_list, int32_t *big_list, int32_t *counts) {
    if (n <= 0) return hipSuccess;
    k_segsort_classify<<<grid_for(n, 256, 65536), 256, 0, st>>>(ptr, n, mid_list, big_list,
                                                                 counts);
    return hipGetLastError();
}

hipError_t launch_segsort_small(hipStream_t st, const int32_t *ptr, int32_t n, int32_t *val) {
    if (n <= 0) return hipSuccess;
    k_segsort_small<<<grid_for(n, 256, 65536), 256, 0, st>>>(ptr, n, val);
    return hipGetLastError();
}

hipError_t launch_segsort_mid(hipStream_t st, const int32_t *ptr, const int32_t *mid_list,
                              const int32_t *counts, int32_t grid, int32_t *val) {
    if (grid <= 0) return hipSuccess;
    k_segsort_mid<<<grid, 256, 0, st>>>(ptr, mid_list, counts, val);
    return hipGetLastError();
}

hipError_t launch_segsort_big_load(hipStream_t st, const int32_t *src, int32_t len, int32_t n2,
                                   int32_t *tmp) {
    k_big_load<<<grid_for(n2, 256, 65536), 256, 0, st>>>(src, len, n2, tmp);
    return hipGetLastError();
}

hipError_t launch_bitonic_step(hipStream_t st, int32_t *tmp, int32_t n2, int32_t k, int32_t j) {
    k_bitonic_step<<<grid_for(n2, 256, 65536), 256, 0, st>>>(tmp, n2, k, j);
    return hipGetLastError();
}

hipError_t launch_segsort_big_store(hipStream_t st, const int32_t *tmp, int32_t len,
                                    int32_t *dst) {
    k_copy<<<grid_for(len, 256, 65536), 256, 0, st>>>(dst, tmp, len);
    return hipGetLastError();
}

hipError_t launch_filter(hipStream_t st, const int32_t *ptrM, const int32_t *itmM, int32_t M,
                         int64_t nnz, const int32_t *ptrI, int32_t s, const int32_t *s_item,
                         int32_t *pos, int32_t *part32, int32_t *ptrS, int32_t *itmS,
                         const int32_t *inv, int32_t *start) {
    if (M <= 0) return hipSuccess;
    if (nnz > 0) {
        k_filter_flags<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(itmM, nnz, ptrI, s, s_item, pos);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // in place: every scan thread reads its inputs before writing them
    hipError_t e = launch_scan_i32(st, pos, nnz, pos, part32);
    if (e != hipSuccess) return e;
    k_filter_scatter<<<grid_for(std::max<int64_t>(nnz, (int64_t)M + 1), 256, 65536), 256, 0, st>>>(
        itmM, nnz, pos, ptrM, M, ptrS, itmS, inv, start);
    return hipGetLastError();
}

hipError_t launch_cost(hipStream_t st, const int32_t *ptrI, const int32_t *memI, int32_t N,
                       int32_t s, const int32_t *s_item, const int32_t *ptrS, const int32_t *itmS,
                       int64_t *cost, int32_t *start, int64_t *totals, int32_t full,
                       int32_t have_start) {
    if (N <= 0) return hipSuccess;
    k_cost<<<grid_for((int64_t)N * kWave, 256, 4096), 256, 0, st>>>(
        ptrI, memI, N, s, s_item, ptrS, itmS, cost, start, totals, full, have_start);
    return hipGetLastError();
}

hipError_t launch_mark_lookup(hipStream_t st, const int32_t *ptrI, const int32_t *memI, int32_t N,
                              int32_t s, const int32_t *s_item, int32_t s_max,
                              const int32_t *ptrS, int32_t *start, int64_t *cost) {
    if (N <= 0 || s_max <= 1) return hipSuccess;
    k_mark_lookup<<<grid_for((int64_t)N * kWave, 256, 65536), 256, 0, st>>>(
        ptrI, memI, N, s, s_item, ptrS, start, cost);
    return hipGetLastError();
}

}  // namespace sl
