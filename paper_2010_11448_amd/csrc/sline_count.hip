// Counting kernels of libsline for gfx950: for each kept item a, count the
// members it shares with every kept item b > a and emit the pairs with count
// >= s, sorted by b.
//
// Method (Sec. IV-B/IV-C): item a reaches candidate b only through a shared
// member v, by walking the kept items of N_s(v) that follow a (strictly upper
// triangle).  The paper's per-thread `visited` array becomes a counter table
// in LDS, so every candidate is counted once per shared member and its final
// count is the overlap w_ab itself.  Items smaller than s never appear
// (degree-based pruning: they are dropped from the member lists and from the
// task list).
//
// Work units: item a with W_a wedges is cut into P_a tasks covering equal
// sub-ranges of its candidate range (a, N); P_a = ceil(W_a / target), so every
// task carries about the same number of wedges.  A workgroup takes a group of
// up to `group_parts` consecutive tasks of one item and walks them in order,
// keeping for each member v the cursor into N_s(v) in a register: the walk of
// the first range starts at the back-pointer of (a, v) computed with W_a, and
// each range ends where the list reaches the range's upper bound, found by
// reading the list forward (no search).  Tasks are listed in (a, sub-range)
// order, and an exclusive scan of the per-task pair counts places each task's
// output directly in canonical (a, b) order.
//
// Table: one 32-bit LDS word per slot, 0 = empty, for a range [lo, hi):
//   * dense  (hi - lo <= slots): slot = j - lo, the word is the count;
//   * hashed (hi - lo  > slots): the word packs (j - lo + 1) above the low
//     `cb` bits, which hold the count (cb = bit length of |S_a|, so a count
//     never reaches the key field; ranges too wide for the key field are
//     split).  Home slot = (j - lo) * slots / (hi - lo), one v_mul_hi_u32;
//     linear probing forward without wrap-around into `pad` extra slots.
//     The map is monotone, so two candidates out of order in slot order sit
//     in the same run of occupied slots (a cluster): extraction ranks each
//     candidate against its cluster neighbours and writes it to its final
//     position.  A probe that runs off the table marks the range, which is
//     then cleared and split in halves (depth-first, left half first).
//
// Two kernels: k_count_small (one wave per item with W_a <= small_max) and
// k_count_tasks (one workgroup per task group).  Each runs twice: a count pass
// (pairs per task) and, after the exclusive scan of those counts, a fill pass
// writing (a, b, w) at the task's offset.
#include <algorithm>

#include "sline_internal.h"

namespace sl {

namespace {

constexpr int kR = 8;  // member cursors per thread held in registers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t lds_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// first index p in [lo, hi) with arr[p] >= key (arr ascending), hi if none
__device__ __forceinline__ int32_t lower_bound(const int32_t *arr, int32_t lo, int32_t hi,
                                               int32_t key) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if (arr[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct Range {
    int32_t lo;      // first candidate id
    int32_t hi;      // one past the last candidate id
    uint32_t span;   // hi - lo
    uint32_t mul;    // hashed: home = mulhi(j - lo, mul); 0 = dense
    int32_t limit;   // slots in use (home slots + pad when hashed)
    int32_t cb;      // hashed: count bits of a slot word
    uint32_t cmask;  // (1 << cb) - 1
};

__device__ __forceinline__ Range make_range(int32_t lo, int32_t hi, int32_t slots, int32_t pad,
                                            int32_t cb) {
    Range r;
    r.lo = lo;
    r.hi = hi;
    const int64_t span = (int64_t)hi - lo;
    r.span = (uint32_t)span;
    r.cb = cb;
    r.cmask = (1u << cb) - 1u;
    if (span <= slots) {
        r.mul = 0;
        r.limit = (int32_t)span;
    } else {
        r.mul = (uint32_t)(((uint64_t)slots << 32) / (uint64_t)span);
        r.limit = slots + pad;
    }
    return r;
}

// A hashed range whose ids do not fit the key field of a slot word.
__device__ __forceinline__ bool too_wide(const Range &R) {
    return R.mul != 0 && (uint64_t)R.span >= (1ull << (32 - R.cb));
}

// Count one wedge ending at candidate j.  Returns false if the probe ran off
// the table (the caller splits the range).
__device__ __forceinline__ bool tab_add(uint32_t *tab, const Range &R, int32_t j) {
    const uint32_t x = (uint32_t)(j - R.lo);
    if (x >= R.span) return true;  // outside the range: only with unsorted input (SKIP_VALIDATE)
    if (R.mul == 0) {
        atomicAdd(&tab[x], 1u);
        return true;
    }
    const uint32_t tag = (x + 1u) << R.cb;
    for (int32_t p = (int32_t)__umulhi(x, R.mul); p < R.limit; ++p) {
        uint32_t w = lds_load(&tab[p]);
        if (w == 0u) {
            w = atomicCAS(&tab[p], 0u, tag | 1u);
            if (w == 0u) return true;  // inserted with count 1
        }
        if ((w & ~R.cmask) == tag) {
            atomicAdd(&tab[p], 1u);
            return true;
        }
    }
    return false;
}

struct Smem {
    uint32_t *tab;  // table words
    int2 *runs;     // long member runs of the current range
    int32_t *misc;  // [0] run count, [1] overflow, [2] stack depth, [3..] per-wave words
    int2 *stack;    // ranges still to process
};

// One member's walk over [cur, end) of N_s(v) for the range R, one lane:
// reads four entries at a time and stops at the first id >= R.hi.  Returns
// the new cursor.
__device__ __forceinline__ int32_t walk_lane(const int32_t *itmS, int32_t cur, int32_t end,
                                             const Range &R, const Smem &S, bool &ok) {
    int32_t p = cur;
    while (p < end) {
        int32_t j[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) j[q] = (p + q < end) ? itmS[p + q] : INT32_MAX;
        int32_t taken = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (j[q] < R.hi) {
                ok &= tab_add(S.tab, R, j[q]);
                ++taken;
            }
        }
        p += taken;
        if (taken < 4) break;
    }
    return p;
}

// Insert every wedge of item a whose candidate lies in R.  Members with few
// expected candidates in R are walked by their owning lane; the others are
// queued and walked by whole waves, up to 256 entries per step (sized by the
// expected run length).  On return nc[] holds the advanced cursors of the
// thread's members (not yet committed) and misc[1] is set if a probe ran off
// the table.
template <int NT, int RUNCAP>
__device__ __forceinline__ void insert_range(const CountArgs &A, const Smem &S, const Range &R,
                                             int32_t k0, int32_t k1, const int32_t (&cur)[kR],
                                             const int32_t (&end)[kR], int32_t (&nc)[kR]) {
    constexpr int W = NT / kWave;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const float frac = (float)R.span / (float)((int64_t)A.N - R.lo);
    const float light = (float)A.tune.light_len;
    bool ok = true;
    int32_t slot[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        slot[i] = -1;
        nc[i] = cur[i];
        const int32_t k = k0 + (int32_t)threadIdx.x + i * NT;
        if (k < k1 && cur[i] < end[i]) {
            const float est = (float)(end[i] - cur[i]) * frac;
            if (est <= light) {
                nc[i] = walk_lane(A.itmS, cur[i], end[i], R, S, ok);
            } else {
                const int32_t sl = atomicAdd(&S.misc[0], 1);
                if (sl < RUNCAP) {
                    S.runs[sl] = make_int2(cur[i], end[i]);
                    slot[i] = sl;
                } else {
                    nc[i] = walk_lane(A.itmS, cur[i], end[i], R, S, ok);
                }
            }
        }
    }
    // members past the register window: locate the range by binary search
    for (int32_t k = k0 + (int32_t)threadIdx.x + kR * NT; k < k1; k += NT) {
        const int32_t v = A.memI[k];
        const int32_t e0 = A.ptrS[v + 1];
        const int32_t b = lower_bound(A.itmS, A.start[k], e0, R.lo);
        walk_lane(A.itmS, b, e0, R, S, ok);
    }
    __syncthreads();
    const int32_t nrun = min(S.misc[0], RUNCAP);
    for (int32_t h = wid; h < nrun; h += W) {
        const int2 rr = S.runs[h];
        int32_t p = rr.x;
        const int32_t e = rr.y;
        const float est = (float)(e - p) * frac;
        const int32_t nq = min(4, max(1, (int32_t)((est * 1.25f + 16.0f) * (1.0f / kWave)) + 1));
        for (;;) {
            int32_t j[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t idx = p + q * kWave + lane;
                j[q] = (q < nq && idx < e) ? A.itmS[idx] : INT32_MAX;
            }
            int32_t taken = 0;
            bool full = true;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < nq) {
                    const bool in = j[q] < R.hi;
                    const uint64_t bal = __ballot(in);
                    if (in) ok &= tab_add(S.tab, R, j[q]);
                    taken += __popcll(bal);
                    full &= bal == ~0ull;
                }
            }
            p += taken;
            if (!full) break;
        }
        if (lane == 0) S.runs[h].x = p;
    }
    if (!ok) S.misc[1] = 1;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kR; ++i)
        if (slot[i] >= 0) nc[i] = S.runs[slot[i]].x;
}

// Zero table words [0, limit); `tab` is 16-byte aligned.
template <int NT>
__device__ __forceinline__ void tab_clear(uint32_t *tab, int32_t limit) {
    uint4 *t4 = reinterpret_cast<uint4 *>(tab);
    const int32_t n4 = limit >> 2;
    for (int32_t i = threadIdx.x; i < n4; i += NT) t4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int32_t i = (n4 << 2) + threadIdx.x; i < limit; i += NT) tab[i] = 0u;
}

__device__ __forceinline__ uint32_t slot_count(uint32_t w, const Range &R) {
    return R.mul ? (w & R.cmask) : w;
}

// Extract the candidates with count >= s.  Count mode returns their number;
// fill mode also writes (a, b, w) in b order at out + base.  Leaves the table
// cleared.  Returns a block-uniform count.
template <int NT>
__device__ __forceinline__ int32_t tab_extract(const CountArgs &A, const Smem &S, const Range &R,
                                               int32_t a, bool fill, int64_t base) {
    constexpr int W = NT / kWave;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int32_t L = R.limit;
    const int32_t per_wave = ((L + W * kWave - 1) / (W * kWave)) * kWave;
    const int32_t r0 = wid * per_wave;
    const int32_t r1 = min(L, r0 + per_wave);
    const uint32_t s = (uint32_t)A.s;
    int32_t mine = 0;
    for (int32_t i = r0; i < r1; i += kWave) {
        const int32_t slot = i + lane;
        const uint32_t w = slot < r1 ? S.tab[slot] : 0u;
        mine += __popcll(__ballot(slot_count(w, R) >= s));
    }
    if (lane == 0) S.misc[3 + wid] = mine;
    __syncthreads();
    int32_t run = 0, total = 0;
    for (int w = 0; w < W; ++w) {
        const int32_t t = S.misc[3 + w];
        if (w < wid) run += t;
        total += t;
    }
    if (fill && total) {
        for (int32_t i = r0; i < r1; i += kWave) {
            const int32_t slot = i + lane;
            const uint32_t w = slot < r1 ? S.tab[slot] : 0u;
            const uint32_t c = slot_count(w, R);
            const bool q = c >= s;
            const uint64_t bal = __ballot(q);
            if (q) {
                int32_t pos = run + (int32_t)lanes_below(bal);
                int32_t key;
                if (R.mul) {
                    // rank against the cluster around `slot`: entries before it
                    // in the cluster move past it when their key is larger
                    const uint32_t tag = w >> R.cb;
                    int32_t left = 0, less = 0;
                    for (int32_t q2 = slot - 1; q2 >= 0; --q2) {
                        const uint32_t u = S.tab[q2];
                        if (u == 0u) break;
                        if ((u & R.cmask) >= s) {
                            ++left;
                            less += (u >> R.cb) < tag;
                        }
                    }
                    for (int32_t q2 = slot + 1; q2 < L; ++q2) {
                        const uint32_t u = S.tab[q2];
                        if (u == 0u) break;
                        if ((u & R.cmask) >= s && (u >> R.cb) < tag) ++less;
                    }
                    pos += less - left;
                    key = R.lo + (int32_t)tag - 1;
                } else {
                    key = R.lo + slot;
                }
                A.out_a[base + pos] = a;
                A.out_b[base + pos] = key;
                A.out_w[base + pos] = (int32_t)c;
            }
            run += __popcll(bal);
        }
    }
    __syncthreads();
    tab_clear<NT>(S.tab, L);
    __syncthreads();
    return total;
}

// Candidates [lo, hi) of item a with a table of `slots` home slots: insert,
// split on overflow, extract; the member cursors advance to hi.  Returns the
// pairs produced (block-uniform).
template <int NT, int PAD, int RUNCAP>
__device__ __forceinline__ int64_t run_range(const CountArgs &A, const Smem &S, int32_t a,
                                             int32_t lo, int32_t hi, int32_t slots, int32_t cb,
                                             int32_t k0, int32_t k1, int32_t (&cur)[kR],
                                             const int32_t (&end)[kR], bool fill, int64_t base,
                                             int64_t &passes) {
    if (threadIdx.x == 0) {
        S.stack[0] = make_int2(lo, hi);
        S.misc[2] = 1;
    }
    __syncthreads();
    int64_t produced = 0;
    for (;;) {
        // every thread reads the stack before anyone may change it (the next
        // call's thread 0 rewrites it as soon as it leaves this loop)
        const int32_t depth = S.misc[2];
        const int2 top = depth ? S.stack[depth - 1] : make_int2(0, 0);
        __syncthreads();
        if (depth == 0) break;
        if (threadIdx.x == 0) {
            S.misc[2] = depth - 1;
            S.misc[0] = 0;
            S.misc[1] = 0;
        }
        __syncthreads();
        const Range R = make_range(top.x, top.y, slots, PAD, cb);
        bool split = too_wide(R);
        if (!split) {
            int32_t nc[kR];
            insert_range<NT, RUNCAP>(A, S, R, k0, k1, cur, end, nc);
            ++passes;
            split = S.misc[1] != 0;
            if (!split) {
                produced += tab_extract<NT>(A, S, R, a, fill, base + produced);
#pragma unroll
                for (int i = 0; i < kR; ++i) cur[i] = nc[i];
                continue;
            }
            // a probe ran off the table: clear it
            __syncthreads();
            tab_clear<NT>(S.tab, R.limit);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int32_t mid = (int32_t)(((int64_t)top.x + top.y) / 2);
            const int32_t d = S.misc[2];
            S.stack[d] = make_int2(mid, top.y);
            S.stack[d + 1] = make_int2(top.x, mid);
            S.misc[2] = d + 2;
        }
        __syncthreads();
    }
    return produced;
}

// Cursors of the thread's members for a walk starting at candidate lo.
template <int NT>
__device__ __forceinline__ void init_cursors(const CountArgs &A, int32_t a, int32_t lo, int32_t k0,
                                             int32_t k1, int32_t (&cur)[kR], int32_t (&end)[kR]) {
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const int32_t k = k0 + (int32_t)threadIdx.x + i * NT;
        cur[i] = 0;
        end[i] = 0;
        if (k < k1) {
            const int32_t v = A.memI[k];
            const int32_t e = A.ptrS[v + 1];
            int32_t c = A.start[k];
            if (lo > a + 1) c = lower_bound(A.itmS, c, e, lo);
            cur[i] = c;
            end[i] = e;
        }
    }
}

// Count bits for item a: its size bounds every overlap.
__device__ __forceinline__ int32_t count_bits(int32_t size) {
    return 32 - __clz((uint32_t)max(size, 1));
}

// Number of tasks of an item and the sub-range of task p.
__device__ __forceinline__ int32_t task_parts(int64_t cost, int32_t small_max, int32_t target) {
    if (cost <= 0) return 0;
    if (cost <= small_max) return 1;
    return (int32_t)((cost + target - 1) / target);
}

__device__ __forceinline__ void task_range(int32_t a, int32_t N, int32_t p, int32_t P, int32_t &lo,
                                           int32_t &hi) {
    const int64_t first = (int64_t)a + 1, span = (int64_t)N - first;
    lo = (int32_t)(first + span * p / P);
    hi = (int32_t)(first + span * (p + 1) / P);
}

constexpr int kSmallPad = 64;
constexpr int kSmallRunCap = 128;
constexpr int kTaskPad = 64;
constexpr int kTaskRunCap = 512;
constexpr int kStack = 64;

// --------------------------------------------------------------- small

__global__ __launch_bounds__(kWave) void k_count_small(CountArgs A) {
    constexpr int LIM = kSmallSlots + kSmallPad;
    __shared__ __align__(16) uint32_t tab[LIM];
    __shared__ int2 runs[kSmallRunCap];
    __shared__ int2 stack[kStack];
    __shared__ int32_t misc[8];
    const Smem S{tab, runs, misc, stack};
    const bool fill = A.task_off != nullptr;
    tab_clear<kWave>(tab, LIM);
    const int32_t n_small = A.task_counts[0];
    int64_t passes = 0;
    __syncthreads();
    for (int32_t r = blockIdx.x; r < n_small; r += gridDim.x) {
        const int32_t t = A.small_tasks[r];
        const int32_t a = A.task_item[t];
        const int64_t c = A.cost[a];
        // 2 W_a home slots (load <= 1/2), rounded up to whole waves
        int32_t want = (int32_t)std::min<int64_t>(2 * c, kSmallSlots);
        want = std::min(kSmallSlots, std::max(kWave, ((want + kWave - 1) / kWave) * kWave));
        const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
        int32_t cur[kR], end[kR];
        init_cursors<kWave>(A, a, a + 1, k0, k1, cur, end);
        const int64_t base = fill ? A.task_off[t] : 0;
        const int64_t produced = run_range<kWave, kSmallPad, kSmallRunCap>(
            A, S, a, a + 1, A.N, want, count_bits(k1 - k0), k0, k1, cur, end, fill, base, passes);
        if (!fill && threadIdx.x == 0) A.task_cnt[t] = (int32_t)produced;
        __syncthreads();
    }
    if (threadIdx.x == 0 && passes && A.passes)
        atomicAdd((unsigned long long *)A.passes, (unsigned long long)passes);
}

// --------------------------------------------------------------- tasks

__global__ __launch_bounds__(kTaskThreads, 4) void k_count_tasks(CountArgs A) {
    constexpr int NT = kTaskThreads;
    constexpr int LIM = kTaskSlots + kTaskPad;
    __shared__ __align__(16) uint32_t tab[LIM];
    __shared__ int2 runs[kTaskRunCap];
    __shared__ int2 stack[kStack];
    __shared__ int32_t misc[3 + NT / kWave + 1];
    __shared__ int32_t sh_task;
    const Smem S{tab, runs, misc, stack};
    const bool fill = A.task_off != nullptr;
    tab_clear<NT>(tab, LIM);
    const int32_t n_groups = A.task_counts[1];
    int64_t passes = 0;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) sh_task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int32_t r = sh_task;
        __syncthreads();
        if (r >= n_groups) break;
        const int32_t t0 = A.big_tasks[r];
        const int32_t a = A.task_item[t0];
        const int32_t p0 = A.task_part[t0];
        const int32_t P = task_parts(A.cost[a], A.tune.small_max_wedges, A.tune.task_wedges);
        const int32_t p1 = min(P, p0 + A.tune.group_parts);
        const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
        const int32_t cb = count_bits(k1 - k0);
        int32_t lo, hi;
        task_range(a, A.N, p0, P, lo, hi);
        int32_t cur[kR], end[kR];
        init_cursors<NT>(A, a, lo, k0, k1, cur, end);
        for (int32_t q = p0; q < p1; ++q) {
            task_range(a, A.N, q, P, lo, hi);
            const int32_t t = t0 + (q - p0);
            const int64_t base = fill ? A.task_off[t] : 0;
            const int64_t produced = run_range<NT, kTaskPad, kTaskRunCap>(
                A, S, a, lo, hi, kTaskSlots, cb, k0, k1, cur, end, fill, base, passes);
            if (!fill && threadIdx.x == 0) A.task_cnt[t] = (int32_t)produced;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && passes && A.passes)
        atomicAdd((unsigned long long *)A.passes, (unsigned long long)passes);
}

// ----------------------------------------------------------- task lists

__global__ void k_task_count(const int64_t *cost, int32_t N, int32_t small_max, int32_t target,
                             int32_t *ntask) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < N;
         a += (int64_t)gridDim.x * blockDim.x)
        ntask[a] = task_parts(cost[a], small_max, target);
}

// counts[0] small tasks, counts[1] task groups
__global__ void k_task_fill(const int64_t *cost, int32_t N, int32_t small_max, int32_t target,
                            int32_t group, const int64_t *tbase, int32_t *task_item,
                            int32_t *task_part, int32_t *small_tasks, int32_t *groups,
                            int32_t *counts) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < N;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = cost[a];
        const int32_t P = task_parts(c, small_max, target);
        if (P == 0) continue;
        const int64_t t0 = tbase[a];
        for (int32_t p = 0; p < P; ++p) {
            task_item[t0 + p] = (int32_t)a;
            task_part[t0 + p] = p;
        }
        if (c <= small_max) {
            small_tasks[atomicAdd(&counts[0], 1)] = (int32_t)t0;
            continue;
        }
        const int32_t G = (P + group - 1) / group;
        const int32_t at = atomicAdd(&counts[1], G);
        for (int32_t g = 0; g < G; ++g) groups[at + g] = (int32_t)(t0 + (int64_t)g * group);
    }
}

__global__ void k_reset_queue(int32_t *q) { *q = 0; }

inline int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

hipError_t launch_task_count(hipStream_t st, const int64_t *cost, int32_t N, const Tuning &tu,
                             int32_t *ntask) {
    if (N <= 0) return hipSuccess;
    k_task_count<<<grid_for(N, 256, 65536), 256, 0, st>>>(cost, N, tu.small_max_wedges,
                                                         tu.task_wedges, ntask);
    return hipGetLastError();
}

hipError_t launch_task_fill(hipStream_t st, const int64_t *cost, int32_t N, const Tuning &tu,
                            const int64_t *tbase, int32_t *task_item, int32_t *task_part,
                            int32_t *small_tasks, int32_t *big_tasks, int32_t *counts) {
    if (N <= 0) return hipSuccess;
    k_task_fill<<<grid_for(N, 256, 65536), 256, 0, st>>>(cost, N, tu.small_max_wedges,
                                                        tu.task_wedges, std::max(1, tu.group_parts),
                                                        tbase, task_item, task_part, small_tasks,
                                                        big_tasks, counts);
    return hipGetLastError();
}

hipError_t launch_count(hipStream_t st, const CountArgs &A) {
    if (A.N <= 0) return hipSuccess;
    const int gs = std::max(1, A.n_cu * A.tune.small_grid_per_cu);
    k_count_small<<<gs, kWave, 0, st>>>(A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reset_queue<<<1, 1, 0, st>>>(A.queue);
    const int gh = std::max(1, A.n_cu * A.tune.task_grid_per_cu);
    k_count_tasks<<<gh, kTaskThreads, 0, st>>>(A);
    return hipGetLastError();
}

}  // namespace sl
