// Counting kernels of libsline for gfx950: for each kept item a, count the
// members it shares with every kept item b > a and emit the pairs with count
// >= s, sorted by b.
//
// Method (Sec. IV-B/IV-C): item a reaches candidate b only through a shared
// member v, by walking the kept items of N_s(v) that follow a (strictly
// upper triangle).  The paper's per-thread `visited` array becomes a
// per-workgroup counter table in LDS, so every candidate is counted exactly
// once per shared member and its final count is the overlap w_ab itself.
// Items smaller than s never appear (degree-based pruning: they are dropped
// from the member lists and from the item buckets).
//
// Table: `keys`/`cnt` in LDS, addressed by a monotone map of the candidate id
// over the pass range [lo, hi):
//   * dense  (hi - lo <= slots): slot = j - lo, no keys, no probing;
//   * hashed (hi - lo  > slots): home slot = (j - lo) * slots / (hi - lo)
//     (one v_mul_hi_u32), linear probing with wrap-around.  Because the map is
//     monotone, the occupied slots read in order are sorted except inside a
//     run of adjacent occupied slots, and a few odd-even transposition rounds
//     restore the order.
// Passes are sized so that the table never holds more than half its slots
// (distinct candidates <= wedges of the pass), so probing always ends.
//
// Two kernels:
//   * k_count_small: one wave per item with W_a <= small_max; one pass.
//   * k_count_heavy: one 256-thread workgroup per item, items taken from a
//     device work queue in descending W_a order (longest first), the j range
//     cut into passes whose wedge count fits the table; per-member cursors
//     carry the walk from pass to pass.
// Each runs twice: a count pass (pairs per item) and, after the exclusive
// scan of those counts, a fill pass writing (a, b, w) at the item's offset.
#include "sline_internal.h"

namespace sl {

namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int32_t lds_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// first index p in [lo, hi) with arr[p] > key, hi if none
__device__ __forceinline__ int32_t upper_bound(const int32_t *arr, int32_t lo, int32_t hi,
                                               int32_t key) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if (arr[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index p in [lo, hi) with arr[p] >= key, searching outward from lo
__device__ __forceinline__ int32_t gallop_lower(const int32_t *arr, int32_t lo, int32_t hi,
                                                int32_t key) {
    if (lo >= hi || arr[lo] >= key) return lo;
    int32_t prev = lo, step = 1;
    while (prev + step < hi && arr[prev + step] < key) {
        prev += step;
        step <<= 1;
    }
    int32_t l = prev + 1, r = min(prev + step, hi);
    while (l < r) {
        int32_t mid = l + ((r - l) >> 1);
        if (arr[mid] < key) l = mid + 1;
        else r = mid;
    }
    return l;
}

struct Pass {
    int32_t lo;      // first candidate id of the pass
    int32_t slots;   // table slots in use
    uint32_t mul;    // hashed: home = mulhi(j - lo, mul); 0 = dense
    uint32_t range;  // hi - lo (candidates outside are ignored)
};

__device__ __forceinline__ Pass make_pass(int32_t lo, int64_t hi, int32_t max_slots,
                                          int32_t slots_hint) {
    Pass p;
    p.lo = lo;
    const int64_t range = hi - lo;
    p.range = (uint32_t)range;
    if (range <= max_slots) {
        p.slots = (int32_t)range;
        p.mul = 0;
    } else {
        p.slots = slots_hint;
        p.mul = (uint32_t)(((uint64_t)slots_hint << 32) / (uint64_t)range);
    }
    return p;
}

// Add one wedge (a, v, j) to the table.
__device__ __forceinline__ void tab_add(int32_t *keys, int32_t *cnt, const Pass &P, int32_t j,
                                        int32_t *err) {
    const uint32_t x = (uint32_t)(j - P.lo);
    if (x >= P.range) return;  // only reachable with unsorted input under SKIP_VALIDATE
    if (P.mul == 0) {
        atomicAdd(&cnt[x], 1);
        return;
    }
    uint32_t p = __umulhi(x, P.mul);
    for (int32_t probe = 0; probe < P.slots; ++probe) {
        int32_t k = lds_load(&keys[p]);
        if (k == kEmpty) {
            k = atomicCAS(&keys[p], kEmpty, j);
            if (k == kEmpty) k = j;
        }
        if (k == j) {
            atomicAdd(&cnt[p], 1);
            return;
        }
        p = (p + 1 == (uint32_t)P.slots) ? 0u : p + 1;
    }
    atomicOr(err, kErrInternal);
}

// Compact the table entries with count >= s into slots [0, n) in candidate
// order, clear everything else, and return n (block-uniform).  NT threads,
// MAXR = max_slots / NT registers per lane.  When `keep` is false only the
// count is produced and the table is cleared.
template <int NT, int MAXR>
__device__ int32_t tab_extract(int32_t *keys, int32_t *cnt, const Pass &P, int32_t s, bool keep,
                               int32_t *sh_wave /* NT/64 + 1 */) {
    constexpr int W = NT / kWave;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int32_t T = P.slots;
    const int32_t per_wave = ((T + W * kWave - 1) / (W * kWave)) * kWave;
    const int32_t r0 = wid * per_wave;
    int32_t rk[MAXR], rc[MAXR];
    int32_t mine = 0;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        const int32_t slot = r0 + i * kWave + lane;
        int32_t c = 0, k = 0;
        if (i * kWave < per_wave && slot < T) {
            c = cnt[slot];
            if (c >= s) k = P.mul ? keys[slot] : P.lo + slot;
            else c = 0;
        }
        rk[i] = k;
        rc[i] = c;
        mine += __popcll(__ballot(c > 0));
    }
    if (lane == 0) sh_wave[wid] = mine;
    __syncthreads();
    int32_t base = 0, total = 0;
    for (int w = 0; w < W; ++w) {
        const int32_t t = sh_wave[w];
        if (w < wid) base += t;
        total += t;
    }
    // clear the table (everything read is in registers now)
    for (int32_t i = threadIdx.x; i < T; i += NT) {
        cnt[i] = 0;
        if (P.mul) keys[i] = kEmpty;
    }
    __syncthreads();
    if (!keep || total == 0) return total;
    int32_t run = base;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        const bool q = rc[i] > 0;
        const uint64_t bal = __ballot(q);
        if (q) {
            const int32_t pos = run + (int32_t)lanes_below(bal);
            keys[pos] = rk[i];
            cnt[pos] = rc[i];
        }
        run += __popcll(bal);
    }
    __syncthreads();
    if (P.mul) {
        // odd-even transposition until sorted: only adjacent runs can be out of order
        for (;;) {
            int swapped = 0;
            for (int ph = 0; ph < 2; ++ph) {
                for (int32_t i = 2 * threadIdx.x + ph; i + 1 < total; i += 2 * NT) {
                    const int32_t x = keys[i], y = keys[i + 1];
                    if (x > y) {
                        const int32_t cx = cnt[i];
                        keys[i] = y;
                        keys[i + 1] = x;
                        cnt[i] = cnt[i + 1];
                        cnt[i + 1] = cx;
                        swapped = 1;
                    }
                }
                __syncthreads();
            }
            if (!__syncthreads_or(swapped)) break;
        }
    }
    return total;
}

// Write slots [0, n) as pairs (a, keys, cnt) at out + base, then clear them
// (compaction wrote keys in dense passes too).
template <int NT>
__device__ void tab_emit(int32_t *keys, int32_t *cnt, int32_t n, int32_t a, int64_t base,
                         int32_t *oa, int32_t *ob, int32_t *ow) {
    for (int32_t i = threadIdx.x; i < n; i += NT) {
        oa[base + i] = a;
        ob[base + i] = keys[i];
        ow[base + i] = cnt[i];
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += NT) {
        cnt[i] = 0;
        keys[i] = kEmpty;
    }
    __syncthreads();
}

constexpr int kRunCapSmall = 256;
constexpr int kRunCapHeavy = 512;

// --------------------------------------------------------------- small

__global__ __launch_bounds__(kWave) void k_count_small(CountArgs A) {
    __shared__ int32_t keys[kSmallSlots];
    __shared__ int32_t cnt[kSmallSlots];
    __shared__ int2 runs[kRunCapSmall];
    __shared__ int32_t sh_nrun;
    __shared__ int32_t sh_wave[2];
    const int lane = lane_id();
    const bool fill = A.rowoff != nullptr;
    for (int32_t i = lane; i < kSmallSlots; i += kWave) {
        keys[i] = kEmpty;
        cnt[i] = 0;
    }
    const int32_t n_small = A.bins[128];
    __syncthreads();
    for (int32_t r = blockIdx.x; r < n_small; r += gridDim.x) {
        const int32_t a = A.small_list[r];
        const int64_t c = A.cost[a];
        int32_t want = (int32_t)min<int64_t>(2 * c, kSmallSlots);
        want = max(kWave, ((want + kWave - 1) / kWave) * kWave);
        want = min(want, kSmallSlots);
        const Pass P = make_pass(a + 1, A.N, want, want);
        if (lane == 0) sh_nrun = 0;
        __syncthreads();
        const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
        for (int32_t k = k0 + lane; k < k1; k += kWave) {
            const int32_t v = A.memI[k];
            const int32_t e = A.ptrS[v + 1];
            const int32_t b = upper_bound(A.itmS, A.ptrS[v], e, a);
            if (e - b <= A.tune.light_len) {
                for (int32_t p = b; p < e; ++p) tab_add(keys, cnt, P, A.itmS[p], A.err);
            } else {
                const int32_t slot = atomicAdd(&sh_nrun, 1);
                if (slot < kRunCapSmall) runs[slot] = make_int2(b, e);
                else
                    for (int32_t p = b; p < e; ++p) tab_add(keys, cnt, P, A.itmS[p], A.err);
            }
        }
        __syncthreads();
        const int32_t nrun = min(sh_nrun, kRunCapSmall);
        for (int32_t h = 0; h < nrun; ++h) {
            const int2 rr = runs[h];
            for (int32_t p = rr.x + lane; p < rr.y; p += kWave) tab_add(keys, cnt, P, A.itmS[p], A.err);
        }
        __syncthreads();
        const int32_t n = tab_extract<kWave, kSmallSlots / kWave>(keys, cnt, P, A.s, fill, sh_wave);
        if (fill) {
            if (n) tab_emit<kWave>(keys, cnt, n, a, A.rowoff[a], A.out_a, A.out_b, A.out_w);
        } else if (lane == 0) {
            A.rowcnt[a] = n;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- heavy

template <typename T>
__device__ T block_sum(T v, T *sh /* W + 1 */) {
    constexpr int W = kHeavyThreads / kWave;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    T t = 0;
    for (int w = 0; w < W; ++w) t += sh[w];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kHeavyThreads) void k_count_heavy(CountArgs A) {
    constexpr int NT = kHeavyThreads;
    constexpr int W = NT / kWave;
    __shared__ int32_t keys[kHeavySlots];
    __shared__ int32_t cnt[kHeavySlots];
    __shared__ int2 runs[kRunCapHeavy];
    __shared__ int32_t sh_nrun, sh_row;
    __shared__ int32_t sh_wave[W + 1];
    __shared__ int64_t sh_sum[W + 1];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const bool fill = A.rowoff != nullptr;
    for (int32_t i = threadIdx.x; i < kHeavySlots; i += NT) {
        keys[i] = kEmpty;
        cnt[i] = 0;
    }
    const int32_t n_heavy = A.bins[129];
    const int64_t target = (int64_t)kHeavySlots * A.tune.heavy_load_pct / 100;
    int64_t passes = 0;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) sh_row = atomicAdd(A.queue, 1);
        __syncthreads();
        const int32_t r = sh_row;
        __syncthreads();
        if (r >= n_heavy) break;
        const int32_t a = A.heavy_list[r];
        const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
        for (int32_t k = k0 + threadIdx.x; k < k1; k += NT) {
            const int32_t v = A.memI[k];
            A.cur[k] = upper_bound(A.itmS, A.ptrS[v], A.ptrS[v + 1], a);
        }
        int64_t remaining = A.cost[a];
        int64_t x = a + 1;
        int64_t width = max<int64_t>(kHeavySlots, ((int64_t)A.N - x) * target / max<int64_t>(remaining, 1));
        int64_t out_pos = fill ? A.rowoff[a] : 0;
        int64_t n_out = 0;
        while (remaining > 0 && x < A.N) {
            const int64_t hi = min<int64_t>((int64_t)A.N, x + width);
            // wedges of this pass: per member, the run of N_s(v) inside [x, hi)
            int64_t mine = 0;
            for (int32_t k = k0 + threadIdx.x; k < k1; k += NT) {
                const int32_t v = A.memI[k];
                const int32_t c0 = A.cur[k];
                const int32_t e = gallop_lower(A.itmS, c0, A.ptrS[v + 1], (int32_t)hi);
                A.nxt[k] = e;
                mine += e - c0;
            }
            const int64_t E = block_sum<int64_t>(mine, sh_sum);
            if (E > target && hi - x > kHeavySlots) {
                width = max<int64_t>(kHeavySlots, (hi - x) * target / E);
                continue;
            }
            ++passes;
            if (E > 0) {
                const Pass P = make_pass((int32_t)x, hi, kHeavySlots, kHeavySlots);
                if (threadIdx.x == 0) sh_nrun = 0;
                __syncthreads();
                for (int32_t k = k0 + threadIdx.x; k < k1; k += NT) {
                    const int32_t b = A.cur[k], e = A.nxt[k];
                    if (e - b <= A.tune.light_len) {
                        for (int32_t p = b; p < e; ++p) tab_add(keys, cnt, P, A.itmS[p], A.err);
                    } else {
                        const int32_t slot = atomicAdd(&sh_nrun, 1);
                        if (slot < kRunCapHeavy) runs[slot] = make_int2(b, e);
                        else
                            for (int32_t p = b; p < e; ++p) tab_add(keys, cnt, P, A.itmS[p], A.err);
                    }
                }
                __syncthreads();
                const int32_t nrun = min(sh_nrun, kRunCapHeavy);
                for (int32_t h = wid; h < nrun; h += W) {
                    const int2 rr = runs[h];
                    for (int32_t p = rr.x + lane; p < rr.y; p += kWave)
                        tab_add(keys, cnt, P, A.itmS[p], A.err);
                }
                __syncthreads();
                const int32_t n = tab_extract<NT, kHeavySlots / NT>(keys, cnt, P, A.s, fill, sh_wave);
                if (fill && n) {
                    tab_emit<NT>(keys, cnt, n, a, out_pos, A.out_a, A.out_b, A.out_w);
                    out_pos += n;
                }
                n_out += n;
                for (int32_t k = k0 + threadIdx.x; k < k1; k += NT) A.cur[k] = A.nxt[k];
            }
            remaining -= E;
            x = hi;
            width = max<int64_t>(kHeavySlots, E > 0 ? width * target / E : 2 * width);
            __syncthreads();
        }
        if (!fill && threadIdx.x == 0) A.rowcnt[a] = (int32_t)n_out;
        __syncthreads();
    }
    if (threadIdx.x == 0 && passes && A.passes)
        atomicAdd((unsigned long long *)A.passes, (unsigned long long)passes);
}

__global__ void k_reset_queue(int32_t *q) { *q = 0; }

}  // namespace

hipError_t launch_count(hipStream_t st, const CountArgs &A) {
    if (A.N <= 0) return hipSuccess;
    const int gs = max(1, A.n_cu * A.tune.small_grid_per_cu);
    k_count_small<<<gs, kWave, 0, st>>>(A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reset_queue<<<1, 1, 0, st>>>(A.queue);
    const int gh = max(1, A.n_cu * A.tune.heavy_grid_per_cu);
    k_count_heavy<<<gh, kHeavyThreads, 0, st>>>(A);
    return hipGetLastError();
}

}  // namespace sl
