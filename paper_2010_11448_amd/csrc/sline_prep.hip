// Preparation kernels of libsline for gfx950: CSR checks, device-wide
// exclusive scans, the transpose (a stable radix sort of the incidences by
// member), the s-filtered membership lists, the exact per-item wedge count
// W_a and the lookup-only members.
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

// Short rows are walked by groups of kGroup lanes (eight rows per wave);
// longer rows by whole waves, in a second launch that looks at 64 rows at a
// time and takes the long ones in turn.  Short means at most 32 entries.
constexpr int kGroup = 8;

template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int d = W / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <int W>
__device__ __forceinline__ uint64_t group_max(uint64_t v) {
#pragma unroll
    for (int d = W / 2; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Call body(a, gl) for the rows a this launch owns: with W < kWave, every
// row of at most SHORT entries, by a group of W lanes (gl = lane in the
// group); with W == kWave, every longer row, by the whole wave.
template <int W, int SHORT, typename Body>
__device__ __forceinline__ void for_rows(const int32_t *ptrI, int64_t N, Body body) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    if (W < kWave) {
        constexpr int G = kWave / W;
        const int gl = lane & (W - 1);
        for (int64_t a = wave * G + lane / W; a < N; a += nwaves * G) {
            if (ptrI[a + 1] - ptrI[a] > SHORT) continue;  // the whole-wave launch takes it
            body(a, gl);
        }
    } else {
        for (int64_t base = wave * kWave; base < N; base += nwaves * kWave) {
            const int64_t r = base + lane;
            uint64_t m = __ballot(r < N && ptrI[r + 1] - ptrI[r] > SHORT);
            while (m) {
                const int64_t a = base + __builtin_ctzll(m);
                m &= m - 1;
                body(a, lane);
            }
        }
    }
}

__global__ void k_check_rowptr(const int32_t *rp, int32_t m, int32_t *err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && rp[0] != 0) atomicOr(err, kErrRowPtr0);
    if (i < m && rp[i] > rp[i + 1]) atomicOr(err, kErrRowPtrOrder);
}

// One wave per row (grid-stride): the row id of every incidence, member range
// checks and, when asked, the strictly-increasing check of each row.
template <int W>
__global__ __launch_bounds__(256) void k_rows(const int32_t *rp, const int32_t *col, int32_t m,
                                              int32_t n, int64_t nnz, int check_order,
                                              int32_t *rowid, int32_t *err) {
    int32_t bad = 0;
    for_rows<W, 32>(rp, m, [&](int64_t i, int gl) {
        int64_t b = rp[i], e = rp[i + 1];
        if (b < 0) b = 0;
        if (e > nnz) e = nnz;
        for (int64_t k = b + gl; k < e; k += W) {
            int32_t v = col[k];
            rowid[k] = (int32_t)i;
            if (v < 0 || v >= n) bad |= kErrColRange;
            if (check_order && k + 1 < e && col[k + 1] <= v) bad |= kErrColOrder;
        }
    });
    if (bad) atomicOr(err, bad);
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



// start[k] = map[k] + 1 for every item incidence k (lists not filtered: the
// first item after a in N(v) follows a's own position in the list).
__global__ void k_start_from_map(int64_t nnz, const int32_t *map, int32_t *start) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        start[k] = map[k] + 1;
}






// ------------------------------------------------ transpose by radix sort
// The transpose is a stable sort of the incidences (v = col[k], k) by member
// v: least significant digit first, kRsBits bits per pass.  A pass counts
// the digits of each tile of kRsTile keys (k_rs_hist), scans the counts
// bin by bin across tiles, and moves every key to its bin's place
// (k_rs_scatter).  Inside a tile, thread t holds kRsItems consecutive keys
// and counts them per bin in its own LDS counters; a block scan of the
// counters in (bin, thread) order gives every key its place, so equal
// digits keep their order within the tile, and the bin-major offsets keep
// the order of the tiles.
constexpr int kRsBits = 4;
constexpr int kRsBins = 1 << kRsBits;
constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;

// Digit counts of each tile, bin-major: hist[bin * ntiles + tile].
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const int32_t *keys, int64_t n, int shift,
                                                        int32_t *hist, int32_t ntiles) {
    __shared__ int32_t h[kRsBins];
    if (threadIdx.x < kRsBins) h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    int32_t mine = 0;  // lane b < kRsBins: this wave's count of digit b
    for (int i = threadIdx.x & ~(kWave - 1); i < kRsTile; i += kRsThreads) {
        const int64_t p = base + i + lane;
        const int32_t d = p < n ? (int32_t)(((uint32_t)keys[p] >> shift) & (kRsBins - 1)) : -1;
#pragma unroll
        for (int b = 0; b < kRsBins; ++b) {
            const int32_t cb = (int32_t)__popcll(__ballot(d == b));
            if (lane == b) mine += cb;
        }
    }
    if (lane < kRsBins && mine) atomicAdd(&h[lane], mine);
    __syncthreads();
    if (threadIdx.x < kRsBins) hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Move the keys of each tile to their place: off[bin * ntiles + tile] is the
// first output slot of the tile's keys with that digit.  vin null: the value
// of key p is p.  The last pass writes, instead of the values, the final
// maps: kT[q] = value (the incidence), colT[q] = rowid[value] (its item),
// posT[value] = q (kT, posT may be null).
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const int32_t *kin, const int32_t *vin, int64_t n, int shift, const int32_t *off,
    int32_t ntiles, int32_t *kout, int32_t *vout, int32_t last, const int32_t *rowid,
    int32_t *colT, int32_t *kT, int32_t *posT) {
    __shared__ int32_t cnt[kRsBins * kRsThreads];  // [bin][thread]
    __shared__ int32_t sk[kRsTile], sv[kRsTile];   // the tile in sorted order
    __shared__ int32_t sh[kRsThreads / kWave + 1];
    __shared__ int32_t bin_start[kRsBins];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)t * kRsItems;
    int32_t key[kRsItems], val[kRsItems], dig[kRsItems];
#pragma unroll
    for (int b = 0; b < kRsBins; ++b) cnt[b * kRsThreads + t] = 0;
#pragma unroll
    for (int i = 0; i < kRsItems; ++i) {
        const int64_t p = base + i;
        dig[i] = -1;
        if (p < n) {
            key[i] = kin[p];
            val[i] = vin ? vin[p] : (int32_t)p;
            dig[i] = (int32_t)(((uint32_t)key[i] >> shift) & (kRsBins - 1));
            cnt[dig[i] * kRsThreads + t] += 1;
        }
    }
    __syncthreads();
    // exclusive scan of the counters in (bin, thread) order: thread t takes
    // entries [t * kRsBins, (t + 1) * kRsBins) of the flattened array
    int32_t loc[kRsBins];
    int32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kRsBins; ++j) {
        loc[j] = cnt[t * kRsBins + j];
        sum += loc[j];
    }
    int32_t total;
    int32_t run = block_excl_scan<int32_t>(sum, sh, total);
#pragma unroll
    for (int j = 0; j < kRsBins; ++j) {
        cnt[t * kRsBins + j] = run;
        run += loc[j];
    }
    __syncthreads();
    if (t < kRsBins) bin_start[t] = cnt[t * kRsThreads];
    __syncthreads();
    // place the keys in tile order, then write each bin's run with
    // consecutive lanes
#pragma unroll
    for (int i = 0; i < kRsItems; ++i) {
        if (dig[i] < 0) continue;
        const int32_t r = cnt[dig[i] * kRsThreads + t]++;
        sk[r] = key[i];
        sv[r] = val[i];
    }
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
    const int32_t tn = (int32_t)(n - tile0 < kRsTile ? n - tile0 : kRsTile);
    for (int32_t j = t; j < tn; j += kRsThreads) {
        const int32_t k = sk[j], v = sv[j];
        const int32_t b = (int32_t)(((uint32_t)k >> shift) & (kRsBins - 1));
        const int32_t q = off[b * ntiles + blockIdx.x] + (j - bin_start[b]);
        kout[q] = k;
        if (!last) {
            vout[q] = v;
        } else {
            if (kT) kT[q] = v;
            if (posT) posT[v] = q;
            colT[q] = rowid[v];
        }
    }
}

// Row pointers of the transpose from the sorted members: ptr[v] = first slot
// with member >= v, for v = 0..n (members outside [0, n) are clamped; they
// only occur in input that the row checks reject).
__global__ void k_rs_bounds(const int32_t *sk, int64_t nnz, int32_t n, int32_t *ptr) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        int32_t hi = p < nnz ? sk[p] : n;
        int32_t lo = p > 0 ? sk[p - 1] : -1;
        hi = hi < 0 ? 0 : (hi > n ? n : hi);
        lo = lo < -1 ? -1 : (lo > n ? n : lo);
        for (int32_t v = lo + 1; v <= hi; ++v) ptr[v] = (int32_t)p;
    }
}

// -------------------------------------------------------- s filtering

// The s filter as a stream compaction: the filtered lists N_s(v), one after
// the other, are the kept entries of the member lists in their order, so the
// position of a kept entry is the number of kept entries before it.
// kept[it] = 1 if item it has |S| >= s (s_item[it] when given); then
// keep[p] = kept[itmM[p]] for entry p of the member lists (one gather per
// entry instead of the item's two list bounds and its s).
__global__ void k_item_kept(const int32_t *ptrI, int32_t N, int32_t s, const int32_t *s_item,
                            int32_t *kept) {
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < N;
         it += (int64_t)gridDim.x * blockDim.x)
        kept[it] = (ptrI[it + 1] - ptrI[it]) >= (s_item ? s_item[it] : s) ? 1 : 0;
}

__global__ void k_filter_flags(const int32_t *itmM, int64_t nnz, const int32_t *kept,
                               int32_t *keep) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        keep[p] = kept[itmM[p]];
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

// W_a = sum over members v of the number of kept items b > a in N_s(v); 0 for
// items with |S_a| < s.  For every member incidence k of a kept item,
// start[k] = index in itmS of the first item > a in N_s(v) (the back-pointer
// where a's walk over v begins).  totals: kept items, their incidences, W.
template <int W>
__global__ __launch_bounds__(256) void k_cost(const int32_t *ptrI, const int32_t *memI,
                                              int32_t N, int32_t s, const int32_t *s_item,
                                              const int32_t *ptrS, const int32_t *itmS,
                                              int64_t *cost, int32_t *start, int64_t *totals,
                                              int32_t full, int32_t have_start) {
    int64_t kept = 0, kept_nnz = 0, wedges = 0;  // counted by each row's first lane
    for_rows<W, 32>(ptrI, N, [&](int64_t a, int gl) {
        const int32_t b = ptrI[a], e = ptrI[a + 1];
        if (e - b < (s_item ? s_item[a] : s)) {
            if (gl == 0) cost[a] = 0;
            return;
        }
        int64_t c = 0;
        for (int32_t k = b + gl; k < e; k += W) {
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
        c = group_sum<W>(c);
        if (gl == 0) {
            cost[a] = c;
            kept += 1;
            kept_nnz += e - b;
            wedges += c;
        }
    });
    // one atomic per counter and block (same-address atomics serialize)
    kept = wave_sum(kept);
    kept_nnz = wave_sum(kept_nnz);
    wedges = wave_sum(wedges);
    __shared__ int64_t red[3][256 / kWave];
    const int wid = threadIdx.x / kWave;
    if (lane_id() == 0) {
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

// Per kept item: flag as lookup-only the min(s - 1, kMaxLookup) members with
// the most candidates after a (ties to the lower incidence), by setting the
// sign bit of start[k].  At least one member stays unflagged, as |S_a| >= s
// for a kept item.  The item's planning cost becomes the wedges of its
// inserting members (they fill the table), but at least a third of W_a
// (every wedge is still read).  A row of at most W * kKeysPerLane members
// keeps its keys in registers, so the rounds only exchange maxima; longer
// rows read their members again in every round.  The lane that owns
// incidence k is the one that flags it.
constexpr int kKeysPerLane = 4;

template <int W>
__global__ __launch_bounds__(256) void k_mark_lookup(const int32_t *ptrI, const int32_t *memI,
                                                     int32_t N, int32_t s_all,
                                                     const int32_t *s_item, const int32_t *ptrS,
                                                     int32_t *start, int64_t *cost,
                                                     int32_t tiny_max) {
    for_rows<W, kGroup * kKeysPerLane>(ptrI, N, [&](int64_t a, int gl) {
        const int32_t b = ptrI[a], e = ptrI[a + 1];
        const int32_t s = s_item ? s_item[a] : s_all;
        if (e - b < s) return;
        // a tiny item by its exact wedges stays tiny: it is counted one per
        // lane, every wedge, so lookup-only members would change nothing
        if (e - b <= kTinyCap && cost[a] <= tiny_max) return;
        const int32_t rounds = min(min(s - 1, kMaxLookup), e - b - 1);
        int64_t flagged = 0;
        if (e - b <= W * kKeysPerLane) {
            uint64_t key[kKeysPerLane];
#pragma unroll
            for (int i = 0; i < kKeysPerLane; ++i) {
                const int32_t k = b + gl + i * W;
                key[i] = 0;
                if (k < e) {
                    const int32_t st = start[k];
                    const int32_t c = ptrS[memI[k] + 1] - st;
                    if (st >= 0)
                        key[i] = ((uint64_t)(uint32_t)c << 32) | (uint32_t)(INT32_MAX - k);
                }
            }
            for (int32_t r = 0; r < rounds; ++r) {
                uint64_t best = 0;
#pragma unroll
                for (int i = 0; i < kKeysPerLane; ++i) best = key[i] > best ? key[i] : best;
                best = group_max<W>(best);
                if ((best >> 32) == 0) break;  // no member with candidates left
                const int32_t k = INT32_MAX - (int32_t)(uint32_t)best;
#pragma unroll
                for (int i = 0; i < kKeysPerLane; ++i) {
                    if (key[i] == best) {  // keys are distinct: one owner
                        key[i] = 0;
                        start[k] |= (int32_t)0x80000000u;
                    }
                }
                flagged += (int64_t)(best >> 32);
            }
        } else for (int32_t r = 0; r < rounds; ++r) {
            // best unflagged member: most candidates, then lowest k
            uint64_t best = 0;
            for (int32_t k = b + gl; k < e; k += W) {
                const int32_t st = start[k];
                if (st < 0) continue;
                const int32_t c = ptrS[memI[k] + 1] - st;
                const uint64_t key = ((uint64_t)(uint32_t)c << 32) | (uint32_t)(INT32_MAX - k);
                best = key > best ? key : best;
            }
            best = group_max<W>(best);
            if ((best >> 32) == 0) break;  // no member with candidates left
            const int32_t k = INT32_MAX - (int32_t)(uint32_t)best;
            if ((k - b) % W == gl) start[k] |= (int32_t)0x80000000u;
            flagged += (int64_t)(best >> 32);
        }
        if (gl == 0 && flagged) {
            const int64_t w = cost[a];
            cost[a] = max(w - flagged, (w + 2) / 3);
        }
    });
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
    k_rows<kGroup><<<grid_for((int64_t)m * kGroup, 256, 65536), 256, 0, st>>>(
        rp, col, m, n, nnz, check_order, rowid, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_rows<kWave><<<grid_for(m, 256, 4096), 256, 0, st>>>(rp, col, m, n, nnz, check_order, rowid,
                                                         err);
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



hipError_t launch_start_from_map(hipStream_t st, int64_t nnz, const int32_t *map, int32_t *start) {
    if (nnz <= 0) return hipSuccess;
    k_start_from_map<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(nnz, map, start);
    return hipGetLastError();
}







int64_t transpose_tiles(int64_t nnz) { return (nnz + kRsTile - 1) / kRsTile; }

int64_t transpose_hist(int64_t nnz) { return (int64_t)kRsBins * transpose_tiles(nnz) + 1; }

int transpose_passes(int32_t n) {
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
    return std::max(1, (bits + kRsBits - 1) / kRsBits);
}

hipError_t launch_transpose(hipStream_t st, const int32_t *col, int64_t nnz, int32_t n,
                            const int32_t *rowid, int32_t *const rsK[2], int32_t *const rsV[2],
                            int32_t *hist, int32_t *part32, int32_t *ptrT, int32_t *colT,
                            int32_t *kT, int32_t *posT) {
    if (nnz <= 0) return launch_fill_i32(st, ptrT, (int64_t)n + 1, 0);
    const int passes = transpose_passes(n);
    const int32_t ntiles = (int32_t)transpose_tiles(nnz);
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes && e == hipSuccess; ++p) {
        const int32_t *kin = p == 0 ? col : rsK[(p - 1) & 1];
        const int32_t *vin = p == 0 ? nullptr : rsV[(p - 1) & 1];
        const int last = p == passes - 1;
        k_rs_hist<<<ntiles, kRsThreads, 0, st>>>(kin, nnz, p * kRsBits, hist, ntiles);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_scan_i32(st, hist, (int64_t)kRsBins * ntiles, hist, part32);
        if (e == hipSuccess) {
            k_rs_scatter<<<ntiles, kRsThreads, 0, st>>>(kin, vin, nnz, p * kRsBits, hist, ntiles,
                                                       rsK[p & 1], rsV[p & 1], last, rowid, colT,
                                                       kT, posT);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    k_rs_bounds<<<grid_for(nnz + 1, 256, 65536), 256, 0, st>>>(rsK[(passes - 1) & 1], nnz, n,
                                                               ptrT);
    return hipGetLastError();
}

hipError_t launch_filter(hipStream_t st, const int32_t *ptrM, const int32_t *itmM, int32_t M,
                         int64_t nnz, const int32_t *ptrI, int32_t N, int32_t s,
                         const int32_t *s_item, int32_t *kept, int32_t *pos, int32_t *part32,
                         int32_t *ptrS, int32_t *itmS, const int32_t *inv, int32_t *start) {
    if (M <= 0) return hipSuccess;
    if (nnz > 0) {
        k_item_kept<<<grid_for(N, 256, 65536), 256, 0, st>>>(ptrI, N, s, s_item, kept);
        k_filter_flags<<<grid_for(nnz, 256, 65536), 256, 0, st>>>(itmM, nnz, kept, pos);
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
    k_cost<kGroup><<<grid_for((int64_t)N * kGroup, 256, 4096), 256, 0, st>>>(
        ptrI, memI, N, s, s_item, ptrS, itmS, cost, start, totals, full, have_start);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_cost<kWave><<<grid_for(N, 256, 1024), 256, 0, st>>>(
        ptrI, memI, N, s, s_item, ptrS, itmS, cost, start, totals, full, have_start);
    return hipGetLastError();
}

hipError_t launch_mark_lookup(hipStream_t st, const int32_t *ptrI, const int32_t *memI, int32_t N,
                              int32_t s, const int32_t *s_item, int32_t s_max,
                              const int32_t *ptrS, int32_t *start, int64_t *cost,
                              int32_t tiny_max) {
    if (N <= 0 || s_max <= 1) return hipSuccess;
    k_mark_lookup<kGroup><<<grid_for((int64_t)N * kGroup, 256, 65536), 256, 0, st>>>(
        ptrI, memI, N, s, s_item, ptrS, start, cost, tiny_max);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_mark_lookup<kWave><<<grid_for(N, 256, 4096), 256, 0, st>>>(
        ptrI, memI, N, s, s_item, ptrS, start, cost, tiny_max);
    return hipGetLastError();
}

}  // namespace sl
