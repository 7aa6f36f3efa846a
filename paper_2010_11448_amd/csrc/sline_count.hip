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
//     split).  Slots form buckets of four words read with one 16-byte LDS
//     load.  Home bucket = (j - lo) * buckets / (hi - lo), one v_mul_hi_u32;
//     a candidate takes its home bucket or, when that is full, the next
//     bucket with room (no wrap-around; `pad` extra slots at the end).  The
//     map is monotone, so a bucket with a free slot separates smaller from
//     larger candidates: candidates can only be out of order inside a run of
//     full buckets ended by a non-full one (a cluster), and extraction ranks
//     each candidate against its cluster to write it to its final position.
//     A probe that runs off the table marks the range, which is then cleared
//     and split in halves (depth-first, left half first).
//
// Insertion cutoff (s > 1): the members flagged lookup-only (the s - 1
// longest lists of the item, at most kMaxLookup) walk after the others,
// behind a barrier, and only add to keys already in the table: a candidate
// whose overlap reaches s lies in at least one list that inserts it.
//
// Two kernels: k_count_small (one wave per item with W_a <= small_max) and
// k_count_tasks (one workgroup per task group).  Normally one counting pass
// stages every extracted range's (b, w) in a pool and logs where it goes;
// after the exclusive scan of the pairs per task, k_stage_copy moves each
// range to its task's offset, writing (a, b, w).  Tasks that found no room in
// the pool, or every task when no pool could be had, are counted again in a
// fill pass that writes at the task's offset directly.  In product mode
// (`full`, the SpGEMM companion) every b in [0, N) counts, a itself included.
#include <algorithm>
#include <type_traits>

#include "sline_internal.h"

namespace sl {

namespace {

constexpr int kR = 8;        // member cursors per thread held in registers
constexpr int kPiece = 256;  // planned entries per piece of a long member run

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
// Wave index inside the workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

__device__ __forceinline__ int32_t wave_total(int32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
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
    uint32_t mul;    // hashed: home bucket = mulhi(j - lo, mul); 0 = dense
    int32_t limit;   // words in use (home slots + pad when hashed; a multiple of 4)
    int32_t cb;      // hashed: count bits of a slot word
    uint32_t cmask;  // (1 << cb) - 1
    uint32_t psh;    // dense: 2^psh counters per word (4 x 8, 2 x 16 or 1 x 32 bits)
};

// Counters per table word, as a shift, for overlaps of up to 2^cb - 1: four
// 8-bit counters when the item has at most 255 members, two 16-bit ones up
// to 65535, else one.
__device__ __forceinline__ uint32_t pack_shift(int32_t cb) { return cb <= 8 ? 2u : cb <= 16 ? 1u : 0u; }

// Dense ranges (span <= slots << pack_shift(cb)) count candidate j in
// counter j - lo directly: candidate order is counter order, no hashing and
// no overflow (an overlap never exceeds the item's size).  Wider ranges hash.
__device__ __forceinline__ Range make_range(int32_t lo, int32_t hi, int32_t slots, int32_t pad,
                                            int32_t cb) {
    Range r;
    r.lo = lo;
    r.hi = hi;
    const int64_t span = (int64_t)hi - lo;
    r.span = (uint32_t)span;
    r.cb = cb;
    r.cmask = (1u << cb) - 1u;
    r.psh = pack_shift(cb);
    if (span <= ((int64_t)slots << r.psh)) {
        r.mul = 0;
        r.limit = (int32_t)((span + (1 << r.psh) - 1) >> r.psh);
    } else {
        r.psh = 0;
        r.mul = (uint32_t)(((uint64_t)(slots >> 2) << 32) / (uint64_t)span);
        r.limit = slots + pad;
    }
    return r;
}

// A hashed range whose ids do not fit the key field of a slot word.
__device__ __forceinline__ bool too_wide(const Range &R) {
    return R.mul != 0 && (uint64_t)R.span >= (1ull << (32 - R.cb));
}

// The free word a new key takes in a bucket read as (w0..w3): the first free
// one going round from word ws; 4 if the bucket is full.
__device__ __forceinline__ uint32_t free_word(uint32_t ws, uint32_t w0, uint32_t w1, uint32_t w2,
                                              uint32_t w3) {
    const uint32_t f = (w0 == 0u ? 1u : 0u) | (w1 == 0u ? 2u : 0u) | (w2 == 0u ? 4u : 0u) |
                       (w3 == 0u ? 8u : 0u);
    const uint32_t r = ((f | (f << 4)) >> ws) & 15u;
    return r ? ((ws + (uint32_t)__builtin_ctz(r)) & 3u) : 4u;
}

// Hashed insertion of a wedge with key field `tag`, starting at bucket b whose
// contents were read as q.  Returns false if the probe ran off the table.
__device__ __forceinline__ bool tab_probe(uint32_t *tab, const Range &R, uint32_t tag,
                                          uint32_t ws, int32_t b, uint4 q) {
    const uint32_t hmask = ~R.cmask;
    const uint4 *t4 = reinterpret_cast<const uint4 *>(tab);
    const int32_t nb = R.limit >> 2;
    for (;;) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
        int32_t hit = -1;
#pragma unroll
        for (int i = 3; i >= 0; --i)
            if ((w[i] & hmask) == tag) hit = i;
        const uint32_t fw = free_word(ws, q.x, q.y, q.z, q.w);
        const int32_t empty = fw < 4u ? (int32_t)fw : -1;
        if (hit >= 0) {
            atomicAdd(&tab[4 * b + hit], 1u);
            return true;
        }
        if (empty >= 0) {
            const uint32_t old = atomicCAS(&tab[4 * b + empty], 0u, tag | 1u);
            if (old == 0u) return true;  // inserted with count 1
            if ((old & hmask) == tag) {
                atomicAdd(&tab[4 * b + empty], 1u);
                return true;
            }
            // another candidate took the slot: look at this bucket again
        } else if (++b >= nb) {
            return false;  // full bucket without the key: next bucket
        }
        q = t4[b];
    }
}

// Pick word i of a bucket (i in 0..3) without indexing registers dynamically.
__device__ __forceinline__ uint32_t pick4(int32_t i, uint32_t a0, uint32_t a1, uint32_t a2,
                                          uint32_t a3) {
    return i == 0 ? a0 : i == 1 ? a1 : i == 2 ? a2 : a3;
}

// Count up to four wedges (a candidate >= R.hi means none).  The four home
// buckets are read together; every wedge that finds its key there is counted
// with one atomic add and every new key is claimed with one compare-and-swap,
// all four swaps in flight before any result is looked at.  A new key takes
// the first free word going round from its start word, the quarter of its
// bucket's share of the range it falls in: neighbouring entries of a sorted
// list, inserted by neighbouring lanes at once, share a home bucket but
// mostly not a start word, so their swaps do not collide.  Words never become
// free again during a pass, so a key is found in its home bucket or, if that
// bucket was full when it came, in a later one, and a bucket with a free word
// ends any search.  Wedges whose home bucket is full, or whose free word was
// taken by another key meanwhile, finish in the probe loop.
__device__ __forceinline__ bool tab_add4(uint32_t *tab, uint32_t *spare, const Range &R,
                                         int32_t j0, int32_t j1, int32_t j2, int32_t j3) {
    // this lane's spare word: atomics with nothing to count go there, so the
    // atomics need no branches
    uint32_t *const dummy = spare + lane_id();
    const int32_t j[4] = {j0, j1, j2, j3};
    uint32_t x[4];
    bool in[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = (uint32_t)(j[i] - R.lo);
        in[i] = j[i] < R.hi && x[i] < R.span;
    }
    if (R.mul == 0) {
        const uint32_t pm = (1u << R.psh) - 1u, bsh = 5u - R.psh;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            atomicAdd(in[i] ? &tab[x[i] >> R.psh] : dummy, 1u << ((x[i] & pm) << bsh));
        return true;
    }
    const uint32_t hmask = ~R.cmask;
    const uint4 *t4 = reinterpret_cast<const uint4 *>(tab);
    int32_t b[4];
    uint32_t tag[4], ws[4];
    uint4 q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // a wedge outside the range reads bucket 0 and is ignored below
        b[i] = in[i] ? (int32_t)__umulhi(x[i], R.mul) : 0;
        // where the key lies inside its bucket's share of the range
        ws[i] = (x[i] * R.mul) >> 30;
        tag[i] = (x[i] + 1u) << R.cb;
        q[i] = t4[b[i]];
    }
    // first pass: add to a found key, or claim a free word
    uint32_t addr[4], old[4];
    uint32_t pend = 0;  // bit i: wedge i issued a compare-and-swap
    uint32_t slow = 0;  // bit i: wedge i continues in the probe loop
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t w0 = q[i].x, w1 = q[i].y, w2 = q[i].z, w3 = q[i].w;
        const uint32_t fw = free_word(ws[i], w0, w1, w2, w3);
        // same key <=> the words differ only in the count bits (an empty
        // word never matches: the tag is above the count bits)
        int32_t hit = -1;
        if ((w3 ^ tag[i]) <= R.cmask) hit = 3;
        if ((w2 ^ tag[i]) <= R.cmask) hit = 2;
        if ((w1 ^ tag[i]) <= R.cmask) hit = 1;
        if ((w0 ^ tag[i]) <= R.cmask) hit = 0;
        addr[i] = 4u * (uint32_t)b[i] + (hit >= 0 ? (uint32_t)hit : (fw & 3u));
        const bool add = in[i] && hit >= 0;
        const bool cas = in[i] && hit < 0 && fw < 4u;
        const bool full = in[i] && hit < 0 && fw >= 4u;
        atomicAdd(add ? &tab[addr[i]] : dummy, 1u);
        old[i] = atomicCAS(cas ? &tab[addr[i]] : dummy, 0u, tag[i] | 1u);
        pend |= cas ? 1u << i : 0u;
        slow |= full ? 1u << i : 0u;
        b[i] += full ? 1 : 0;  // home bucket full without the key: continue after it
    }
    // second pass: the swaps' results
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool taken = ((pend >> i) & 1u) && old[i] != 0u;
        const bool same = taken && (old[i] & hmask) == tag[i];
        atomicAdd(same ? &tab[addr[i]] : dummy, 1u);
        slow |= (taken && !same) ? 1u << i : 0u;  // another key took the word: look again
    }
    bool ok = true;
    const int32_t nb = R.limit >> 2;
    while (slow) {
        const int32_t i = __builtin_ctz(slow);
        slow &= slow - 1u;
        const int32_t bi = i == 0 ? b[0] : i == 1 ? b[1] : i == 2 ? b[2] : b[3];
        const uint32_t ti = pick4(i, tag[0], tag[1], tag[2], tag[3]);
        const uint32_t wi = pick4(i, ws[0], ws[1], ws[2], ws[3]);
        if (bi >= nb) {
            ok = false;
        } else {
            ok &= tab_probe(tab, R, ti, wi, bi, t4[bi]);
        }
    }
    return ok;
}

// Count up to four wedges whose keys, if present, were inserted before (the
// candidate cannot reach s without them, so an absent key is skipped).  Dense
// ranges add unconditionally: a candidate counted only here stays below s.
__device__ __forceinline__ void tab_look4(uint32_t *tab, const Range &R, int32_t j0, int32_t j1,
                                          int32_t j2, int32_t j3) {
    const int32_t j[4] = {j0, j1, j2, j3};
    uint32_t x[4];
    bool in[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = (uint32_t)(j[i] - R.lo);
        in[i] = j[i] < R.hi && x[i] < R.span;
    }
    if (R.mul == 0) {
        const uint32_t pm = (1u << R.psh) - 1u, bsh = 5u - R.psh;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (in[i]) atomicAdd(&tab[x[i] >> R.psh], 1u << ((x[i] & pm) << bsh));
        return;
    }
    const uint4 *t4 = reinterpret_cast<const uint4 *>(tab);
    const int32_t nb = R.limit >> 2;
    uint32_t tag[4];
    int32_t b[4];
    uint4 q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        tag[i] = (x[i] + 1u) << R.cb;
        b[i] = in[i] ? (int32_t)__umulhi(x[i], R.mul) : 0;
        q[i] = in[i] ? t4[b[i]] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!in[i]) continue;
        for (;;) {
            const uint32_t w0 = q[i].x, w1 = q[i].y, w2 = q[i].z, w3 = q[i].w;
            const bool h0 = (w0 ^ tag[i]) <= R.cmask, h1 = (w1 ^ tag[i]) <= R.cmask;
            const bool h2 = (w2 ^ tag[i]) <= R.cmask, h3 = (w3 ^ tag[i]) <= R.cmask;
            if (h0 || h1 || h2 || h3) {
                atomicAdd(&tab[4 * b[i] + (h0 ? 0 : h1 ? 1 : h2 ? 2 : 3)], 1u);
                break;
            }
            // a bucket with a free word ends the search: the key is absent
            if (w0 == 0u || w1 == 0u || w2 == 0u || w3 == 0u || ++b[i] >= nb) break;
            q[i] = t4[b[i]];
        }
    }
}

struct Smem {
    uint32_t *tab;       // table words
    int2 *runs;          // long member runs of the current range
    int32_t *taken;      // per run: entries of the run inside the current range
    int32_t *misc;       // see kMisc*
    int2 *stack;         // ranges still to process
    uint32_t *spare;     // one word per lane, past the table (targets of idle atomics)
    uint64_t *pool_cur;  // [next, end) of this workgroup's pool chunk
    int32_t *log_cur;    // [next, end) of this workgroup's log chunk
};

// misc words: run pieces, overflow flag, stack depth, staging reservation
// (ok, offset low, offset high), then one word per wave.
constexpr int kMiscRuns = 0, kMiscOverflow = 1, kMiscDepth = 2, kMiscStageOk = 3,
              kMiscStageLo = 4, kMiscStageHi = 5, kMiscWave = 6;

// One member's walk over [cur, end) of N_s(v) for the range R, one lane:
// reads four entries at a time and stops at the first id >= R.hi.  Returns
// the new cursor.
__device__ __forceinline__ int32_t walk_lane(const int32_t *itmS, int32_t cur, int32_t end,
                                             const Range &R, const Smem &S, bool look, bool &ok) {
    int32_t p = cur;
    while (p < end) {
        const int32_t j0 = itmS[p];
        const int32_t j1 = (p + 1 < end) ? itmS[p + 1] : INT32_MAX;
        const int32_t j2 = (p + 2 < end) ? itmS[p + 2] : INT32_MAX;
        const int32_t j3 = (p + 3 < end) ? itmS[p + 3] : INT32_MAX;
        if (look) tab_look4(S.tab, R, j0, j1, j2, j3);
        else ok &= tab_add4(S.tab, S.spare, R, j0, j1, j2, j3);
        const int32_t taken = (j0 < R.hi) + (j1 < R.hi) + (j2 < R.hi) + (j3 < R.hi);
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
                                             const int32_t (&end)[kR], uint32_t lookm, bool look,
                                             int32_t nend, int32_t (&nc)[kR]) {
    constexpr int W = NT / kWave;
    const int lane = lane_id(), wid = wave_id();
    const float frac = (float)R.span / (float)((int64_t)nend - R.lo);
    const float light_len = (float)A.tune.light_len;
    bool ok = true;
    uint32_t light = 0;  // bit i: member i is walked by this lane
    int32_t slot[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        slot[i] = -1;
        if (!look) nc[i] = cur[i];
    }
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const int32_t k = k0 + (int32_t)threadIdx.x + i * NT;
        if (k < k1 && cur[i] < end[i] && (((lookm >> i) & 1u) != 0u) == look) {
            const float est = (float)(end[i] - cur[i]) * frac;
            int32_t sl = -1;
            if (est > light_len) {
                // K pieces of 256 planned entries (the last one open-ended)
                const int32_t K = min(16, (int32_t)((est * 1.25f + 16.0f) * (1.0f / kPiece)) + 1);
                const int32_t s0 = atomicAdd(&S.misc[kMiscRuns], K);
                if (s0 + K <= RUNCAP) {
                    for (int32_t k = 0; k < K; ++k) {
                        const int32_t b = cur[i] + k * kPiece;
                        S.runs[s0 + k] = make_int2(b, k == K - 1 ? end[i] : min(end[i], b + kPiece));
                        S.taken[s0 + k] = 0;
                    }
                    sl = s0 | (K << 16);
                } else {
                    // no room: blank the slots this reservation holds, walk by
                    // lane.  A blank piece is empty and its clamped index
                    // (end - 1) lies in the member's own run.
                    for (int32_t k = s0; k < min(s0 + K, RUNCAP); ++k)
                        S.runs[k] = make_int2(end[i], end[i]);
                }
            }
            if (sl < 0) light |= 1u << i;
            slot[i] = sl;
        }
    }
    // members walked by their own lane, one at a time (one copy of the walk)
    while (light) {
        const uint32_t bit = light & (0u - light);  // lowest member still to walk
        light ^= bit;
        int32_t c = 0, e = 0;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            c = (bit & (1u << r)) ? cur[r] : c;
            e = (bit & (1u << r)) ? end[r] : e;
        }
        const int32_t n = walk_lane(A.itmS, c, e, R, S, look, ok);
#pragma unroll
        for (int r = 0; r < kR; ++r) nc[r] = (bit & (1u << r)) ? n : nc[r];
    }
    // members past the register window: locate the range by binary search
    for (int32_t k = k0 + (int32_t)threadIdx.x + kR * NT; k < k1; k += NT) {
        const int32_t st = A.start[k];
        // dense ranges count every member in one pass (lookup-only ones too)
        if (R.mul != 0 && (st < 0) != look) continue;
        const int32_t v = A.memI[k];
        const int32_t e0 = A.ptrS[v + 1];
        const int32_t b = lower_bound(A.itmS, st & kStartMask, e0, R.lo);
        walk_lane(A.itmS, b, e0, R, S, look, ok);
    }
    __syncthreads();
    // Pieces: each wave keeps four in flight (one 64-entry load each per
    // step), taking pieces h = wid, wid + W, ... in turn.  The entries below
    // R.hi form a prefix of a member's run, so the pieces' counts add up to it.
    const int32_t npiece = __builtin_amdgcn_readfirstlane(min(S.misc[kMiscRuns], RUNCAP));
    int32_t next = wid;
    int32_t pr[4], pp[4], pe[4], pg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pr[k] = -1;
    for (;;) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (pr[k] < 0 && next < npiece) {
                const int2 rr = S.runs[next];
                pr[k] = next;
                pp[k] = __builtin_amdgcn_readfirstlane(rr.x);
                pe[k] = __builtin_amdgcn_readfirstlane(rr.y);
                pg[k] = 0;
                next += W;
            }
            any |= pr[k] >= 0;
        }
        if (!any) break;
        int32_t j[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            j[k] = INT32_MAX;
            if (pr[k] >= 0) {
                // the clamped index lies in the piece's member run: pe - 1 is
                // its last entry, also for empty pieces (blank, or planned
                // past the run's end), which read it and count nothing
                const int32_t v = A.itmS[min(pp[k] + lane, pe[k] - 1)];
                if (pp[k] + lane < pe[k]) j[k] = v;
            }
        }
        if (look) tab_look4(S.tab, R, j[0], j[1], j[2], j[3]);
        else ok &= tab_add4(S.tab, S.spare, R, j[0], j[1], j[2], j[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (pr[k] < 0) continue;
            const int32_t n = __popcll(__ballot(j[k] < R.hi));
            pg[k] += n;
            pp[k] += kWave;
            if (n < kWave || pp[k] >= pe[k]) {
                if (lane == 0 && pg[k]) S.taken[pr[k]] = pg[k];
                pr[k] = -1;
            }
        }
    }
    if (!ok) S.misc[kMiscOverflow] = 1;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        if (slot[i] >= 0) {
            const int32_t s0 = slot[i] & 0xffff, K = slot[i] >> 16;
            int32_t t = S.runs[s0].x;
            for (int32_t k = 0; k < K; ++k) t += S.taken[s0 + k];
            nc[i] = t;
        }
    }
}

// Where the pairs of item `item` at combined output position `pos` go: the
// single output, or (batches written per graph) the arrays of the item's
// graph at the position inside it, ids to be written less `shift`.
struct OutDst {
    int32_t *a, *b, *w;
    int64_t base;
    int32_t shift;
};

__device__ __forceinline__ OutDst out_dst(const CountArgs &A, int32_t item, int64_t pos) {
    OutDst d{A.out_a, A.out_b, A.out_w, pos, 0};
    const int32_t G = A.n_graphs;
    if (G > 0) {
        int32_t lo = 0, hi = G;  // g_ibase[lo] <= item < g_ibase[hi]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (A.g_ibase[mid] <= item) lo = mid;
            else hi = mid;
        }
        d.shift = (int32_t)A.g_ibase[lo];
        if (A.g_out) {
            d.a = A.g_out[lo];
            d.b = A.g_out[G + lo];
            d.w = A.g_out[2 * G + lo];
            d.base = pos - A.g_off[lo];
        }
    }
    return d;
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

// Counters >= s of one word of a packed dense range (2^psh counters of
// 32 >> psh bits each).
__device__ __forceinline__ int32_t packed_hits(uint32_t w, uint32_t psh, uint32_t s) {
    if (psh == 2u)
        return ((w & 0xffu) >= s) + (((w >> 8) & 0xffu) >= s) + (((w >> 16) & 0xffu) >= s) +
               ((w >> 24) >= s);
    return ((w & 0xffffu) >= s) + ((w >> 16) >= s);
}

// Pairs (counters >= s) in the bucket of four words q.
__device__ __forceinline__ int32_t bucket_pairs(const uint4 &q, const Range &R, uint32_t s) {
    if (R.psh == 0u)
        return (slot_count(q.x, R) >= s) + (slot_count(q.y, R) >= s) + (slot_count(q.z, R) >= s) +
               (slot_count(q.w, R) >= s);
    return packed_hits(q.x, R.psh, s) + packed_hits(q.y, R.psh, s) + packed_hits(q.z, R.psh, s) +
           packed_hits(q.w, R.psh, s);
}

// Sum over the wave of n (0 <= n < 32) and the sum over the lanes below this
// one, from the ballots of its bits (nb = bits of n that can be set).
__device__ __forceinline__ void wave_bits_prefix(int32_t n, int nb, int32_t &before, int32_t &step) {
    before = 0;
    step = 0;
    for (int b = 0; b < nb; ++b) {
        const uint64_t m = __ballot((n >> b) & 1);
        before += (int32_t)lanes_below(m) << b;
        step += (int32_t)__popcll(m) << b;
    }
}

__device__ __forceinline__ void cswap(uint32_t &x, uint32_t &y) {
    const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
    x = lo;
    y = hi;
}

__device__ __forceinline__ bool bucket_full(const uint4 &q) {
    return q.x != 0u && q.y != 0u && q.z != 0u && q.w != 0u;
}

// Stage mode, thread 0 of a workgroup: room for `total` pairs in the pool and
// `nrec` consecutive log records, taken from this workgroup's chunks (one
// global atomic per new chunk; records of a chunk left unused stay zero, i.e.
// empty).  Returns false if the pool or the log has no room left.
__device__ __forceinline__ bool stage_reserve(const CountArgs &A, uint64_t *pool_cur,
                                              int32_t *log_cur, int32_t total, int32_t nrec,
                                              uint64_t &off, int32_t &rec) {
    off = pool_cur[0];
    rec = 0;
    if (off + (uint64_t)total > pool_cur[1]) {
        const uint64_t size = max((uint64_t)total, (uint64_t)A.pool_chunk);
        off = atomicAdd(A.pool_head, (unsigned long long)size);
        if (off + size <= (uint64_t)A.pool_cap) {
            pool_cur[1] = off + size;
        } else if (off + (uint64_t)total <= (uint64_t)A.pool_cap) {
            pool_cur[1] = (uint64_t)A.pool_cap;
        } else {
            pool_cur[1] = 0;
            return false;
        }
    }
    pool_cur[0] = off + (uint64_t)total;
    if (log_cur[0] + nrec > log_cur[1]) {
        const int32_t size = max(nrec, A.log_chunk);
        const int32_t r = atomicAdd(A.log_head, size);
        log_cur[0] = r;
        log_cur[1] = (int32_t)min((int64_t)r + size, (int64_t)A.log_cap);
    }
    rec = log_cur[0];
    if (rec + nrec > log_cur[1]) return false;
    log_cur[0] = rec + nrec;
    return true;
}

// Extract the candidates with count >= s and return their number
// (block-uniform).  Each lane holds one bucket (four slots, one 16-byte LDS
// read), so the order inside a bucket is settled in registers; only buckets
// in a run of full buckets (or right after one) rank their entries against
// the neighbouring buckets of the run.  Fill mode writes (a, b, w) in b order
// at task_off[t] + rel; stage mode reserves room in the pool, writes (b, w)
// there and logs the range (or flags task t when the pool or the log is
// full).  Leaves the table cleared.
template <int NT, int RUNCAP>
__device__ __forceinline__ int32_t tab_extract(const CountArgs &A, const Smem &S, const Range &R,
                                               int32_t a, int32_t sa, int32_t t, int64_t rel) {
    constexpr int W = NT / kWave;
    // each wave lists the buckets of its block that hold pairs, in order, in
    // the run arrays (idle during extraction): LCAP 16-bit entries per wave
    constexpr int LCAP = (int)(RUNCAP * sizeof(int2) / sizeof(uint16_t)) / W;
    const int lane = lane_id(), wid = wave_id();
    const int32_t L = R.limit;
    const int32_t nbk = (L + 3) >> 2;  // words past L are zero
    const int32_t per_wave = ((nbk + W * kWave - 1) / (W * kWave)) * kWave;
    const int32_t b0 = wid * per_wave;
    const int32_t b1 = min(nbk, b0 + per_wave);
    const uint32_t s = (uint32_t)sa;
    const uint4 *t4 = reinterpret_cast<const uint4 *>(S.tab);
    uint16_t *const lst = reinterpret_cast<uint16_t *>(S.runs) + wid * LCAP;
    __syncthreads();  // the insertion has finished reading the run arrays
    // bits of a bucket's pair count: up to 4 pairs, or 16 with packed counters
    const int nbits = R.psh ? 5 : 3;
    int32_t mine = 0, nact = 0;
    for (int32_t i = b0; i < b1; i += kWave) {
        const int32_t bk = i + lane;
        const uint4 q = bk < b1 ? t4[bk] : make_uint4(0u, 0u, 0u, 0u);
        const int32_t n = bucket_pairs(q, R, s);
        int32_t nb_before, nb_step;
        wave_bits_prefix(n, nbits, nb_before, nb_step);
        mine += nb_step;
        const uint64_t am = __ballot(n > 0);
        const int32_t slot = nact + (int32_t)lanes_below(am);
        if (n > 0 && slot < LCAP) lst[slot] = (uint16_t)bk;
        nact += (int32_t)__popcll(am);
    }
    if (lane == 0) S.misc[kMiscWave + wid] = mine;
    __syncthreads();
    int32_t run = 0, total = 0;
    for (int w = 0; w < W; ++w) {
        const int32_t tw = S.misc[kMiscWave + w];
        if (w < wid) run += tw;
        total += tw;
    }
    bool write = false;
    int64_t base = 0;
    int32_t shift = 0;  // fill mode, batches written per graph: the graph's item base
    int32_t *dst_a = nullptr, *dst_b = nullptr, *dst_w = nullptr;
    if (total && A.mode == kModeFill) {
        write = true;
        const OutDst od = out_dst(A, a, A.task_off[t] + rel);
        base = od.base;
        shift = od.shift;
        dst_a = od.a;
        dst_b = od.b;
        dst_w = od.w;
    } else if (total && A.mode == kModeStage) {
        if (threadIdx.x == 0) {
            uint64_t off;
            int32_t rec;
            const bool ok = stage_reserve(A, S.pool_cur, S.log_cur, total, 1, off, rec);
            if (ok) {
                StageRec r;
                r.off = (int64_t)off;
                r.t = t;
                r.rel = (int32_t)rel;
                r.n = total;
                r.pad = 0;
                A.log[rec] = r;
            } else if (atomicExch(&A.need[t], 1) == 0) {
                atomicAdd(A.need_count, 1);
            }
            S.misc[kMiscStageOk] = ok ? 1 : 0;
            S.misc[kMiscStageLo] = (int32_t)(uint32_t)(off & 0xffffffffull);
            S.misc[kMiscStageHi] = (int32_t)(uint32_t)(off >> 32);
        }
        __syncthreads();
        if (S.misc[kMiscStageOk]) {
            write = true;
            base = (int64_t)(((uint64_t)(uint32_t)S.misc[kMiscStageHi] << 32) |
                             (uint64_t)(uint32_t)S.misc[kMiscStageLo]);
            dst_b = A.pool_b;
            dst_w = A.pool_w;
        }
    }
    if (write) {
        // One bucket per lane (bk, valid when vb): its pairs go to
        // run + (pairs of this wave's buckets before it).  `listed`: the
        // lanes hold the listed buckets, not consecutive ones.
        bool prev_full = R.mul && b0 > 0 && b0 < b1 && bucket_full(t4[b0 - 1]);
        auto emit = [&](auto listed, int32_t bk, bool vb) {
            const uint4 q = vb ? t4[bk] : make_uint4(0u, 0u, 0u, 0u);
            const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
            uint32_t c[4];
            bool ok[4];
            int32_t n = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[k] = slot_count(wv[k], R);
                ok[k] = c[k] >= s;
                n += ok[k];
            }
            if (R.psh) n = bucket_pairs(q, R, s);
            // exclusive prefix of n over the lanes
            int32_t before, step;
            wave_bits_prefix(n, nbits, before, step);
            if (R.mul == 0 && R.psh) {
                // packed dense: counter order is candidate order
                const uint32_t per = 1u << R.psh, cbits = 32u >> R.psh;
                const uint32_t cm = (cbits == 32u) ? 0xffffffffu : ((1u << cbits) - 1u);
                int32_t pos = run + before;
                for (int k = 0; k < 4 && n; ++k) {
                    for (uint32_t j = 0; j < per; ++j) {
                        const uint32_t cnt = (wv[k] >> (j * cbits)) & cm;
                        if (cnt >= s) {
                            const int32_t b = R.lo + (int32_t)(((uint32_t)(4 * bk + k) << R.psh) + j);
                            if (dst_a) dst_a[base + pos] = a - shift;
                            dst_b[base + pos] = b - shift;
                            if (dst_w) dst_w[base + pos] = (int32_t)cnt;
                            ++pos;
                        }
                    }
                }
            } else if (R.mul == 0) {
                // dense: slot order is candidate order
                int32_t pos = run + before;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (ok[k]) {
                        if (dst_a) dst_a[base + pos] = a - shift;
                        dst_b[base + pos] = R.lo + 4 * bk + k - shift;
                        if (dst_w) dst_w[base + pos] = (int32_t)c[k];
                        ++pos;
                    }
                }
            } else {
                // the bucket's kept words in candidate order (a word orders
                // like its key, which sits above the count bits; words not
                // kept sort last): five compare-exchanges
                uint32_t key[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) key[k] = ok[k] ? wv[k] : 0xFFFFFFFFu;
                cswap(key[0], key[1]);
                cswap(key[2], key[3]);
                cswap(key[0], key[2]);
                cswap(key[1], key[3]);
                cswap(key[1], key[2]);
                uint32_t tag[4];
                int32_t rank[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    tag[k] = key[k] >> R.cb;
                    rank[k] = k;
                }
                // runs of full buckets: a bucket ends a run unless it is full
                const bool full = bucket_full(q) && vb;
                bool pf;  // the bucket before this one is full
                if (decltype(listed)::value) {
                    pf = vb && bk > 0 && bucket_full(t4[bk - 1]);
                } else {
                    const uint64_t fm = __ballot(full);
                    pf = lane ? ((fm >> (lane - 1)) & 1ull) != 0 : prev_full;
                    prev_full = ((fm >> 63) & 1ull) != 0;
                }
                int32_t left = 0;
                if (n && (full || pf)) {
                    // full buckets before this one in the same run
                    for (int32_t b2 = bk - 1; b2 >= 0; --b2) {
                        const uint4 lv = t4[b2];
                        if (!bucket_full(lv)) break;
                        const uint32_t l[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
                        for (int k2 = 0; k2 < 4; ++k2) {
                            if ((l[k2] & R.cmask) >= s) {
                                ++left;
                                const uint32_t tg = l[k2] >> R.cb;
#pragma unroll
                                for (int k = 0; k < 4; ++k) rank[k] += tg < tag[k];
                            }
                        }
                    }
                    // buckets after this one up to the first that is not full
                    bool more = full;
                    for (int32_t b2 = bk + 1; more && b2 < nbk; ++b2) {
                        const uint4 rv = t4[b2];
                        more = bucket_full(rv);
                        const uint32_t r[4] = {rv.x, rv.y, rv.z, rv.w};
#pragma unroll
                        for (int k2 = 0; k2 < 4; ++k2) {
                            if ((r[k2] & R.cmask) >= s) {
                                const uint32_t tg = r[k2] >> R.cb;
#pragma unroll
                                for (int k = 0; k < 4; ++k) rank[k] += tg < tag[k];
                            }
                        }
                    }
                }
                const int32_t pos = run + before - left;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (k < n) {
                        const int32_t p = pos + rank[k];
                        if (dst_a) dst_a[base + p] = a - shift;
                        dst_b[base + p] = R.lo + (int32_t)tag[k] - 1 - shift;
                        if (dst_w) dst_w[base + p] = (int32_t)(key[k] & R.cmask);
                    }
                }
            }
            run += step;
        };
        if (nact <= LCAP) {
            // only the buckets that hold pairs, 64 at a time
            for (int32_t i = 0; i < nact; i += kWave) {
                const bool vb = i + lane < nact;
                emit(std::true_type{}, vb ? (int32_t)lst[i + lane] : 0, vb);
            }
        } else {
            for (int32_t i = b0; i < b1; i += kWave)
                emit(std::false_type{}, i + lane, i + lane < b1);
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
                                             int32_t sa, int32_t nend, int32_t t, int32_t lo,
                                             int32_t hi, int32_t slots,
                                             int32_t cb, int32_t k0, int32_t k1, int32_t (&cur)[kR],
                                             const int32_t (&end)[kR], uint32_t lookm,
                                             int64_t &passes) {
    if (threadIdx.x == 0) {
        S.stack[0] = make_int2(lo, hi);
        S.misc[kMiscDepth] = 1;
    }
    __syncthreads();
    int64_t produced = 0;
    for (;;) {
        // every thread reads the stack before anyone may change it (the next
        // call's thread 0 rewrites it as soon as it leaves this loop)
        const int32_t depth = S.misc[kMiscDepth];
        const int2 top = depth ? S.stack[depth - 1] : make_int2(0, 0);
        __syncthreads();
        if (depth == 0) break;
        if (threadIdx.x == 0) {
            S.misc[kMiscDepth] = depth - 1;
            S.misc[kMiscRuns] = 0;
            S.misc[kMiscOverflow] = 0;
        }
        __syncthreads();
        const Range R = make_range(top.x, top.y, slots, PAD, cb);
        bool split = too_wide(R);
        if (!split) {
            int32_t nc[kR];
            // a dense range has room for every candidate: all members count in
            // one pass, lookup-only ones included
            const uint32_t lm = R.mul ? lookm : 0u;
            insert_range<NT, RUNCAP>(A, S, R, k0, k1, cur, end, lm, false, nend, nc);
            ++passes;
            split = S.misc[kMiscOverflow] != 0;
            if (!split && sa > 1 && R.mul != 0) {
                // members marked lookup-only count candidates the others inserted
                __syncthreads();
                if (threadIdx.x == 0) S.misc[kMiscRuns] = 0;
                __syncthreads();
                insert_range<NT, RUNCAP>(A, S, R, k0, k1, cur, end, lm, true, nend, nc);
            }
            if (!split) {
                produced += tab_extract<NT, RUNCAP>(A, S, R, a, sa, t, produced);
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
            const int32_t d = S.misc[kMiscDepth];
            S.stack[d] = make_int2(mid, top.y);
            S.stack[d + 1] = make_int2(top.x, mid);
            S.misc[kMiscDepth] = d + 2;
        }
        __syncthreads();
    }
    return produced;
}

// Cursors of the thread's members for a walk starting at candidate lo.
template <int NT>
__device__ __forceinline__ void init_cursors(const CountArgs &A, int32_t a, int32_t lo, int32_t k0,
                                             int32_t k1, int32_t (&cur)[kR], int32_t (&end)[kR],
                                             uint32_t &lookm) {
    lookm = 0;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const int32_t k = k0 + (int32_t)threadIdx.x + i * NT;
        cur[i] = 0;
        end[i] = 0;
        if (k < k1) {
            const int32_t v = A.memI[k];
            const int32_t e = A.ptrS[v + 1];
            const int32_t st = A.start[k];
            lookm |= (uint32_t)(st < 0) << i;
            int32_t c = st & kStartMask;
            if (lo > (A.full ? 0 : a + 1)) c = lower_bound(A.itmS, c, e, lo);
            cur[i] = c;
            end[i] = e;
        }
    }
}

// Count bits for item a: its size bounds every overlap.
__device__ __forceinline__ int32_t count_bits(int32_t size) {
    return 32 - __clz((uint32_t)max(size, 1));
}

// Number of tasks of an item: P = ceil(cost / target) equal sub-ranges of
// its candidate range of `span` ids, each about `target` wedges.  When the
// item's candidates are dense enough -- at least dense_min wedges (by the
// planning cost) on average in each sub-range narrow enough for its packed
// dense counters (slots << pack_shift(size)) -- the item is cut into that many
// sub-ranges instead (if more): counting one of them costs an add per wedge
// and an in-order scan, with no hashing.  dense_min = 0 keeps P as is.
__device__ __forceinline__ int32_t task_parts(int64_t cost, int32_t small_max, int32_t target,
                                              int64_t span, int32_t size, int32_t dense_min,
                                              int32_t slots) {
    if (cost <= 0) return 0;
    if (cost <= small_max) return 1;
    int64_t P = (cost + target - 1) / target;
    if (dense_min > 0 && span > 0) {
        const int64_t cap = (int64_t)slots << pack_shift(32 - __clz((uint32_t)max(size, 1)));
        const int64_t Pd = (span + cap - 1) / cap;
        if (Pd > P && cost >= (int64_t)dense_min * Pd) P = Pd;
    }
    return (int32_t)min(P, (int64_t)INT32_MAX);
}

// Candidate span of item a: [a + 1, end) (product mode: [0, end)), end = its
// graph's end (batches) or N.
__device__ __forceinline__ int64_t item_span(const int32_t *item_end, int32_t N, int32_t full,
                                             int32_t a) {
    const int64_t e = item_end ? item_end[a] : N;
    return e - (full ? 0 : (int64_t)a + 1);
}

// Sub-range p of P of the candidate range [first, N) of an item.
__device__ __forceinline__ void task_range(int32_t first_id, int32_t N, int32_t p, int32_t P,
                                           int32_t &lo, int32_t &hi) {
    const int64_t first = first_id, span = (int64_t)N - first;
    lo = (int32_t)(first + span * p / P);
    hi = (int32_t)(first + span * (p + 1) / P);
}

constexpr int kSmallPad = 64;
constexpr int kSmallRunCap = 128;
constexpr int kTaskPad = 64;
constexpr int kTaskRunCap = 256;
constexpr int kStack = 64;

// A counting launch with nothing to do: the plan's bounds were exceeded (or
// its input is malformed), or a fill pass that only recounts tasks flagged in
// `need` while none is flagged.
__device__ __forceinline__ bool count_idle(const CountArgs &A) {
    if (A.abort && *A.abort != 0) return true;
    return A.mode == kModeFill && A.need && A.need_count && *A.need_count == 0;
}

// --------------------------------------------------------------- small

// SLOTS: home slots of the wave's table (Tuning::small_slots).
template <int SLOTS>
__global__ __launch_bounds__(kWave) void k_count_small(CountArgs A) {
    constexpr int LIM = SLOTS + kSmallPad;
    __shared__ __align__(16) uint32_t tab[LIM + kWave];
    __shared__ int2 runs[kSmallRunCap];
    __shared__ int32_t taken[kSmallRunCap];
    __shared__ int2 stack[kStack];
    __shared__ int32_t misc[kMiscWave + 1];
    __shared__ uint64_t pool_cur[2];
    __shared__ int32_t log_cur[2];
    const Smem S{tab, runs, taken, misc, stack, tab + LIM, pool_cur, log_cur};
    if (count_idle(A)) return;  // uniform: every thread reads the same words
    if (threadIdx.x == 0) {
        pool_cur[0] = pool_cur[1] = 0;
        log_cur[0] = log_cur[1] = 0;
    }
    tab_clear<kWave>(tab, LIM);
    const int32_t n_small = A.task_counts[0];
    int64_t passes = 0;
    __syncthreads();
    for (int32_t r = blockIdx.x; r < n_small; r += gridDim.x) {
        const int32_t t = A.small_tasks[r];
        if (A.mode == kModeFill && A.need && !A.need[t]) continue;
        const int32_t a = A.small_items[r];
        const int64_t c = A.cost[a];
        // 2 W_a home slots (load <= 1/2), rounded up to whole waves
        int32_t want = (int32_t)std::min<int64_t>(2 * c, SLOTS);
        want = std::min(SLOTS, std::max(kWave, ((want + kWave - 1) / kWave) * kWave));
        const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
        int32_t cur[kR], end[kR];
        uint32_t lookm;
        const int32_t nend = A.item_end ? A.item_end[a] : A.N;
        init_cursors<kWave>(A, a, A.full ? 0 : a + 1, k0, k1, cur, end, lookm);
        const int64_t produced = run_range<kWave, kSmallPad, kSmallRunCap>(
            A, S, a, A.s_item ? A.s_item[a] : A.s, nend, t, A.full ? 0 : a + 1, nend, want,
            count_bits(k1 - k0), k0, k1, cur, end, lookm, passes);
        if (A.mode != kModeFill && threadIdx.x == 0) A.task_cnt[t] = (int32_t)produced;
        __syncthreads();
    }
    if (threadIdx.x == 0 && passes && A.passes)
        atomicAdd((unsigned long long *)A.passes, (unsigned long long)passes);
}

// --------------------------------------------------------------- tiny

// One lane per tiny item: a single-task item with a planning cost of at most
// Tuning::tiny_max_wedges (so at most kTinyCap wedges, the planning cost
// being at least a third of them) and at most kTinyCap members, outside
// product mode.  The lane copies the candidates of all its members' walks
// into its own column of an LDS buffer, sorts them, and counts each run of
// equal ids: that count is the overlap.  The candidates come out ascending,
// in output order.  A workgroup stages the pairs of its 256 items with one
// reservation.
__global__ __launch_bounds__(kTinyThreads) void k_count_tiny(CountArgs A) {
    constexpr int NT = kTinyThreads;
    __shared__ int32_t buf[kTinyCap * NT];  // column of lane i: buf[q * NT + i]
    __shared__ int32_t red[2][NT / kWave];
    __shared__ uint64_t pool_cur[2];
    __shared__ int32_t log_cur[2];
    __shared__ int32_t res[4];  // ok, offset low, offset high, first record
    if (count_idle(A)) return;
    if (threadIdx.x == 0) {
        pool_cur[0] = pool_cur[1] = 0;
        log_cur[0] = log_cur[1] = 0;
    }
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    int32_t *col = buf + tid;
    const int32_t n_tiny = A.task_counts[2];
    __syncthreads();
    for (int32_t base = blockIdx.x * NT; base < n_tiny; base += gridDim.x * NT) {
        const int32_t r = base + tid;
        bool act = r < n_tiny;
        int32_t t = 0, a = 0, nc = 0, np = 0, sa = 1;
        if (act) {
            t = A.tiny_tasks[r];
            a = A.tiny_items[r];
            if (A.mode == kModeFill && A.need && !A.need[t]) act = false;
        }
        if (act) {
            sa = A.s_item ? A.s_item[a] : A.s;
            const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
            for (int32_t k = k0; k < k1; ++k) {
                const int32_t v = A.memI[k];
                const int32_t e = A.ptrS[v + 1];
                for (int32_t p = A.start[k] & kStartMask; p < e; ++p) {
                    if (nc == kTinyCap) {
                        atomicOr(A.err, kErrInternal);  // the planning bound was wrong
                        break;
                    }
                    col[nc * NT] = A.itmS[p];
                    ++nc;
                }
            }
            // insertion sort of the lane's column
            for (int32_t i = 1; i < nc; ++i) {
                const int32_t x = col[i * NT];
                int32_t j = i - 1;
                while (j >= 0 && col[j * NT] > x) {
                    col[(j + 1) * NT] = col[j * NT];
                    --j;
                }
                col[(j + 1) * NT] = x;
            }
            for (int32_t i = 0; i < nc;) {
                int32_t j = i + 1;
                while (j < nc && col[j * NT] == col[i * NT]) ++j;
                np += (j - i) >= sa;
                i = j;
            }
        }
        if (act && A.mode != kModeFill) A.task_cnt[t] = np;
        // where this lane's pairs go
        int32_t *dst_a = nullptr, *dst_b = nullptr, *dst_w = nullptr;
        int64_t at = 0;
        int32_t shift = 0;
        if (A.mode == kModeFill) {
            if (act && np) {
                const OutDst od = out_dst(A, a, A.task_off[t]);
                dst_a = od.a;
                dst_b = od.b;
                dst_w = od.w;
                at = od.base;
                shift = od.shift;
            }
        } else if (A.mode == kModeStage) {
            // pairs and records before this lane in the workgroup
            int32_t pb, pstep;
            wave_bits_prefix(np, 6, pb, pstep);
            const uint64_t hm = __ballot(np > 0);
            if (lane == 0) {
                red[0][wid] = pstep;
                red[1][wid] = (int32_t)__popcll(hm);
            }
            __syncthreads();
            int32_t pbefore = pb, rbefore = (int32_t)lanes_below(hm), total = 0, nrec = 0;
            for (int w = 0; w < NT / kWave; ++w) {
                if (w < wid) {
                    pbefore += red[0][w];
                    rbefore += red[1][w];
                }
                total += red[0][w];
                nrec += red[1][w];
            }
            if (tid == 0) {
                uint64_t off = 0;
                int32_t rec = 0;
                const bool ok = total > 0 && stage_reserve(A, pool_cur, log_cur, total, nrec, off, rec);
                res[0] = ok ? 1 : 0;
                res[1] = (int32_t)(uint32_t)(off & 0xffffffffull);
                res[2] = (int32_t)(uint32_t)(off >> 32);
                res[3] = rec;
            }
            __syncthreads();
            if (act && np) {
                if (res[0]) {
                    const int64_t off = (int64_t)(((uint64_t)(uint32_t)res[2] << 32) |
                                                  (uint64_t)(uint32_t)res[1]);
                    at = off + pbefore;
                    dst_b = A.pool_b;
                    dst_w = A.pool_w;
                    StageRec rec;
                    rec.off = at;
                    rec.t = t;
                    rec.rel = 0;
                    rec.n = np;
                    rec.pad = 0;
                    A.log[res[3] + rbefore] = rec;
                } else if (atomicExch(&A.need[t], 1) == 0) {
                    atomicAdd(A.need_count, 1);  // counted again by the fill pass
                }
            }
            __syncthreads();  // res and red are rewritten by the next round
        }
        if (dst_b) {
            int32_t q = 0;
            for (int32_t i = 0; i < nc;) {
                int32_t j = i + 1;
                const int32_t b = col[i * NT];
                while (j < nc && col[j * NT] == b) ++j;
                if (j - i >= sa) {
                    if (dst_a) dst_a[at + q] = a - shift;
                    dst_b[at + q] = b - shift;
                    if (dst_w) dst_w[at + q] = j - i;
                    ++q;
                }
                i = j;
            }
        }
    }
}

// --------------------------------------------------------------- tasks

// SLOTS: home slots of the workgroup's table (Tuning::task_slots); MINB:
// waves per SIMD the register budget is planned for (the table's LDS allows
// no more); NT: threads per workgroup.
template <int SLOTS, int MINB, int NT>
__global__ __launch_bounds__(NT, MINB) void k_count_tasks(CountArgs A) {
    constexpr int LIM = SLOTS + kTaskPad;
    __shared__ __align__(16) uint32_t tab[LIM + kWave];
    __shared__ int2 runs[kTaskRunCap];
    __shared__ int32_t taken[kTaskRunCap];
    __shared__ int2 stack[kStack];
    __shared__ int32_t misc[kMiscWave + NT / kWave];
    __shared__ int32_t sh_task;
    __shared__ uint64_t pool_cur[2];
    __shared__ int32_t log_cur[2];
    const Smem S{tab, runs, taken, misc, stack, tab + LIM, pool_cur, log_cur};
    if (count_idle(A)) return;  // uniform: every thread reads the same words
    if (threadIdx.x == 0) {
        pool_cur[0] = pool_cur[1] = 0;
        log_cur[0] = log_cur[1] = 0;
    }
    tab_clear<NT>(tab, LIM);
    const int32_t n_groups = A.task_counts[1];
    int64_t passes = 0;
    int64_t my_wedges = 0, my_nnz = 0, my_pairs = 0;
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
        const int32_t P = task_parts(A.cost[a], A.tune.small_max_wedges, A.tune.task_wedges,
                                     item_span(A.item_end, A.N, A.full, a),
                                     A.ptrI[a + 1] - A.ptrI[a], A.tune.dense_min_wedges,
                                     SLOTS);
        const int32_t p1 = min(P, p0 + A.tune.group_parts);
        const int32_t k0 = A.ptrI[a], k1 = A.ptrI[a + 1];
        const int32_t cb = count_bits(k1 - k0);
        const int32_t sa = A.s_item ? A.s_item[a] : A.s;
        const int32_t nend = A.item_end ? A.item_end[a] : A.N;
        int32_t cur[kR], end[kR];
        uint32_t lookm = 0;
        bool fresh = true;  // cursors must be placed at the range start
        for (int32_t q = p0; q < p1; ++q) {
            int32_t lo, hi;
            task_range(A.full ? 0 : a + 1, nend, q, P, lo, hi);
            const int32_t t = t0 + (q - p0);
            if (A.mode == kModeFill && A.need && !A.need[t]) {
                fresh = true;
                continue;
            }
            if (fresh) {
                init_cursors<NT>(A, a, lo, k0, k1, cur, end, lookm);
                if (q == 0 && A.mode != kModeFill) {
                    // work figures of this kernel: the item's incidences and wedges
#pragma unroll
                    for (int i = 0; i < kR; ++i) my_wedges += end[i] - cur[i];
                    for (int32_t k = k0 + (int32_t)threadIdx.x + kR * NT; k < k1; k += NT)
                        my_wedges += A.ptrS[A.memI[k] + 1] - (A.start[k] & kStartMask);
                    my_nnz += k1 - k0;
                }
            }
            fresh = false;
            const int64_t produced = run_range<NT, kTaskPad, kTaskRunCap>(
                A, S, a, sa, nend, t, lo, hi, SLOTS, cb, k0, k1, cur, end, lookm, passes);
            if (A.mode != kModeFill && threadIdx.x == 0) {
                A.task_cnt[t] = (int32_t)produced;
                my_pairs += produced;
            }
        }
        __syncthreads();
    }
    if (A.passes && A.mode != kModeFill) {
        // one atomic per counter and workgroup (same-address atomics serialize)
        unsigned long long *wk = (unsigned long long *)A.passes;
        int64_t w = my_wedges;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) w += __shfl_xor(w, d, kWave);
        __shared__ int64_t red[NT / kWave];
        if (lane_id() == 0) red[threadIdx.x / kWave] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int i = 0; i < NT / kWave; ++i) t += red[i];
            if (t) atomicAdd(&wk[2], (unsigned long long)t);
            if (my_nnz) atomicAdd(&wk[1], (unsigned long long)my_nnz);
            if (my_pairs) atomicAdd(&wk[3], (unsigned long long)my_pairs);
        }
    }
    if (threadIdx.x == 0 && passes && A.passes)
        atomicAdd((unsigned long long *)A.passes, (unsigned long long)passes);
}

// ----------------------------------------------------------- task lists

// What task_parts needs to know about the items besides their cost.
struct PlanItems {
    const int32_t *ptrI;      // item lists (sizes)
    const int32_t *item_end;  // per item: end of its graph's items (batches), or null
    int32_t full;             // product mode
    int32_t dense_min;        // Tuning::dense_min_wedges
    int32_t slots;            // Tuning::task_slots
};

__device__ __forceinline__ int32_t plan_parts(const PlanItems &I, const int64_t *cost, int32_t N,
                                              int32_t small_max, int32_t target, int32_t a) {
    return task_parts(cost[a], small_max, target, item_span(I.item_end, N, I.full, a),
                      I.ptrI[a + 1] - I.ptrI[a], I.dense_min, I.slots);
}

__global__ void k_task_count(const int64_t *cost, int32_t N, int32_t small_max, int32_t target,
                             PlanItems I, int32_t *ntask) {
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < N;
         a += (int64_t)gridDim.x * blockDim.x)
        ntask[a] = plan_parts(I, cost, N, small_max, target, (int32_t)a);
}

// counts[0] small tasks, counts[1] task groups
// Each workgroup fills the tasks of a contiguous chunk of items.  The slots
// of the two lists are claimed with one global atomic per list and workgroup
// (same-address atomics serialize), then handed out inside the workgroup
// with LDS atomics, one per wave and step.
__global__ __launch_bounds__(256) void k_task_fill(const int64_t *cost, int32_t N,
                                                   int32_t small_max, int32_t target,
                                                   int32_t tiny_max, PlanItems I,
                                                   int32_t group, const int64_t *tbase,
                                                   int32_t *task_item, int32_t *task_part,
                                                   int32_t *small_tasks, int32_t *small_items,
                                                   int32_t *tiny_tasks, int32_t *tiny_items,
                                                   int32_t *groups, int32_t *counts,
                                                   int32_t chunk, const int32_t *abort) {
    if (abort && *abort != 0) return;
    __shared__ int32_t sh[3];
    const int lane = lane_id();
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < N ? lo + chunk : N;
    if (threadIdx.x == 0) sh[0] = sh[1] = sh[2] = 0;
    __syncthreads();
    // a tiny item: one task, a planning cost of at most tiny_max and at most
    // kTinyCap members, outside product mode (see k_count_tiny)
    auto is_tiny = [&](int64_t a, int64_t c) {
        return c <= tiny_max && !I.full && I.ptrI[a + 1] - I.ptrI[a] <= kTinyCap;
    };
    // pass 1: list entries of the chunk
    int32_t ns = 0, ng = 0, nt = 0;
    for (int64_t a = lo + threadIdx.x; a < hi; a += blockDim.x) {
        const int64_t c = cost[a];
        const int32_t P = plan_parts(I, cost, N, small_max, target, (int32_t)a);
        if (P == 0) continue;
        if (c <= small_max) {
            if (is_tiny(a, c)) ++nt;
            else ++ns;
        } else {
            ng += (P + group - 1) / group;
        }
    }
    ns = wave_total(ns);
    ng = wave_total(ng);
    nt = wave_total(nt);
    if (lane == 0) {
        if (ns) atomicAdd(&sh[0], ns);
        if (ng) atomicAdd(&sh[1], ng);
        if (nt) atomicAdd(&sh[2], nt);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sh[0] = sh[0] ? atomicAdd(&counts[0], sh[0]) : 0;
        sh[1] = sh[1] ? atomicAdd(&counts[1], sh[1]) : 0;
        sh[2] = sh[2] ? atomicAdd(&counts[2], sh[2]) : 0;
    }
    __syncthreads();
    // pass 2: tasks, and the list entries at the claimed slots
    for (int64_t base = lo + (threadIdx.x & ~(kWave - 1)); base < hi; base += blockDim.x) {
        const int64_t a = base + lane;
        int64_t c = 0;
        int32_t P = 0;
        int64_t t0 = 0;
        if (a < hi) {
            c = cost[a];
            P = plan_parts(I, cost, N, small_max, target, (int32_t)a);
            if (P > 0) t0 = tbase[a];
        }
        for (int32_t p = 0; p < P; ++p) {
            task_item[t0 + p] = (int32_t)a;
            task_part[t0 + p] = p;
        }
        const bool one = P > 0 && c <= small_max;
        const bool tiny = one && is_tiny(a, c);
        const bool small = one && !tiny;
        const int32_t G = (P > 0 && !one) ? (P + group - 1) / group : 0;
        const uint64_t sm = __ballot(small), tm = __ballot(tiny);
        int32_t sbase = 0, tbase0 = 0;
        if (lane == 0 && sm) sbase = atomicAdd(&sh[0], (int32_t)__popcll(sm));
        if (lane == 0 && tm) tbase0 = atomicAdd(&sh[2], (int32_t)__popcll(tm));
        sbase = __shfl(sbase, 0, kWave);
        tbase0 = __shfl(tbase0, 0, kWave);
        if (small) {
            const int32_t q = sbase + (int32_t)lanes_below(sm);
            small_tasks[q] = (int32_t)t0;
            small_items[q] = (int32_t)a;
        }
        if (tiny) {
            const int32_t q = tbase0 + (int32_t)lanes_below(tm);
            tiny_tasks[q] = (int32_t)t0;
            tiny_items[q] = (int32_t)a;
        }
        int32_t incl = G;  // inclusive prefix of G over the wave
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t u = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += u;
        }
        const int32_t tot = __shfl(incl, kWave - 1, kWave);
        int32_t gbase = 0;
        if (lane == kWave - 1 && tot) gbase = atomicAdd(&sh[1], tot);
        gbase = __shfl(gbase, kWave - 1, kWave);
        const int32_t at = gbase + incl - G;
        for (int32_t g = 0; g < G; ++g) groups[at + g] = (int32_t)(t0 + (int64_t)g * group);
    }
}

__global__ void k_reset_queue(int32_t *q) { *q = 0; }

// One wave per staged range (grid-stride): pool -> final (a, b, w).
// A record as the stage pass wrote it, checked all the same: it guards the
// indices the copy uses.
__device__ __forceinline__ bool stage_rec_ok(const CountArgs &A, const StageRec &rec) {
    return rec.t >= 0 && rec.t < A.n_tasks && rec.n >= 0 && rec.off >= 0 &&
           rec.off + rec.n <= A.pool_cap;
}

// Records of at most this many pairs are copied by one lane each (a task of a
// tiny or small item stages a handful of pairs); longer ones by a whole wave.
constexpr int32_t kLaneRec = 32;

__global__ __launch_bounds__(256) void k_stage_copy(CountArgs A, int32_t n_rec) {
    if (A.abort && *A.abort != 0) return;
    if (n_rec < 0) n_rec = min(*A.log_head, A.log_cap);
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    // short records: one lane each
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rec;
         r += (int64_t)gridDim.x * blockDim.x) {
        const StageRec rec = A.log[r];
        if (rec.n > kLaneRec) continue;  // a wave's, below
        if (!stage_rec_ok(A, rec)) {
            atomicOr(A.err, kErrInternal);
            continue;
        }
        if (rec.n == 0 || A.need[rec.t]) continue;
        const int32_t a = A.task_item[rec.t];
        const int64_t dst = A.task_off[rec.t] + rec.rel;
        if (rec.rel < 0 || dst + rec.n > A.task_off[rec.t + 1]) {
            atomicOr(A.err, kErrInternal);
            continue;
        }
        const OutDst od = out_dst(A, a, dst);
        for (int32_t i = 0; i < rec.n; ++i) {
            od.a[od.base + i] = a - od.shift;
            od.b[od.base + i] = A.pool_b[rec.off + i] - od.shift;
            if (od.w) od.w[od.base + i] = A.pool_w[rec.off + i];
        }
    }
    // long records: one wave each
    for (int64_t r = wave; r < n_rec; r += nwaves) {
        const StageRec rec = A.log[r];
        if (rec.n <= kLaneRec) continue;  // copied above
        if (!stage_rec_ok(A, rec)) {
            if (lane == 0) atomicOr(A.err, kErrInternal);
            continue;
        }
        if (A.need[rec.t]) continue;
        const int32_t a = A.task_item[rec.t];
        const int64_t dst = A.task_off[rec.t] + rec.rel;
        if (rec.rel < 0 || dst + rec.n > A.task_off[rec.t + 1]) {
            if (lane == 0) atomicOr(A.err, kErrInternal);
            continue;
        }
        const OutDst od = out_dst(A, a, dst);
        // four loads per lane in flight before the stores
        for (int32_t i0 = 0; i0 < rec.n; i0 += 4 * kWave) {
            int32_t bv[4], wv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t i = i0 + u * kWave + lane;
                bv[u] = 0;
                wv[u] = 0;
                if (i < rec.n) {
                    bv[u] = A.pool_b[rec.off + i];
                    if (od.w) wv[u] = A.pool_w[rec.off + i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t i = i0 + u * kWave + lane;
                if (i < rec.n) {
                    od.a[od.base + i] = a - od.shift;
                    od.b[od.base + i] = bv[u] - od.shift;
                    if (od.w) od.w[od.base + i] = wv[u];
                }
            }
        }
    }
}

inline int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

hipError_t launch_task_count(hipStream_t st, const int64_t *cost, int32_t N, const Tuning &tu,
                             const int32_t *ptrI, const int32_t *item_end, int32_t full,
                             int32_t *ntask) {
    if (N <= 0) return hipSuccess;
    const PlanItems I{ptrI, item_end, full, tu.dense_min_wedges, tu.task_slots};
    k_task_count<<<grid_for(N, 256, 65536), 256, 0, st>>>(cost, N, tu.small_max_wedges,
                                                         tu.task_wedges, I, ntask);
    return hipGetLastError();
}

hipError_t launch_task_fill(hipStream_t st, const int64_t *cost, int32_t N, const Tuning &tu,
                            const int32_t *ptrI, const int32_t *item_end, int32_t full,
                            const int64_t *tbase, int32_t *task_item, int32_t *task_part,
                            int32_t *small_tasks, int32_t *small_items, int32_t *tiny_tasks,
                            int32_t *tiny_items, int32_t *big_tasks, int32_t *counts,
                            const int32_t *abort) {
    if (N <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(1024, ((int64_t)N + 255) / 256);
    const int32_t chunk = (int32_t)((((int64_t)N + blocks - 1) / blocks + 255) / 256 * 256);
    const int64_t grid = ((int64_t)N + chunk - 1) / chunk;
    const PlanItems I{ptrI, item_end, full, tu.dense_min_wedges, tu.task_slots};
    k_task_fill<<<(unsigned)grid, 256, 0, st>>>(cost, N, tu.small_max_wedges, tu.task_wedges,
                                                tu.tiny_max_wedges, I,
                                                std::max(1, tu.group_parts), tbase, task_item,
                                                task_part, small_tasks, small_items, tiny_tasks,
                                                tiny_items, big_tasks, counts, chunk, abort);
    return hipGetLastError();
}

hipError_t launch_count(hipStream_t st, const CountArgs &A, hipEvent_t mid) {
    if (A.N <= 0) return hipSuccess;
    if (A.tune.tiny_max_wedges > 0 && !A.full) {
        // LDS (the 32 KB candidate buffer) allows four workgroups per CU
        k_count_tiny<<<std::max(1, A.n_cu * 4), kTinyThreads, 0, st>>>(A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int gs = std::max(1, A.n_cu * A.tune.small_grid_per_cu);
    switch (A.tune.small_slots) {
    case 512: k_count_small<512><<<gs, kWave, 0, st>>>(A); break;
    case 2048: k_count_small<2048><<<gs, kWave, 0, st>>>(A); break;
    default: k_count_small<1024><<<gs, kWave, 0, st>>>(A); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reset_queue<<<1, 1, 0, st>>>(A.queue);
    if (mid) {
        e = hipEventRecord(mid, st);
        if (e != hipSuccess) return e;
    }
    const int gh = std::max(1, A.n_cu * A.tune.task_grid_per_cu);
    switch (A.tune.task_slots) {
    case 4480: k_count_tasks<4480, 4, 256><<<gh, 256, 0, st>>>(A); break;
    case 13440: k_count_tasks<13440, 2, 256><<<gh, 256, 0, st>>>(A); break;
    // twice the table and twice the threads: two workgroups per CU keep
    // four waves per SIMD, as four of 256 threads do
    case 17920: k_count_tasks<17920, 4, 512><<<gh, 512, 0, st>>>(A); break;
    default: k_count_tasks<8960, 4, 256><<<gh, 256, 0, st>>>(A); break;
    }
    return hipGetLastError();
}

hipError_t launch_stage_copy(hipStream_t st, const CountArgs &A, int32_t n_rec) {
    if (n_rec == 0 || (n_rec < 0 && A.log_cap <= 0)) return hipSuccess;
    const int64_t most = n_rec < 0 ? A.log_cap : n_rec;
    k_stage_copy<<<grid_for(most * kWave, 256, 16384), 256, 0, st>>>(A, n_rec);
    return hipGetLastError();
}

}  // namespace sl
