// Internal declarations shared by the host side and the device kernels of
// libsline.  Not installed; the public interface is include/sline.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sl {

constexpr int kWave = 64;
constexpr int32_t kEmpty = -1;

// Error bits accumulated on the device while checking the input CSR.
enum : int32_t {
    kErrRowPtr0 = 1,      // row_ptr[0] != 0
    kErrRowPtrOrder = 2,  // row_ptr decreases
    kErrColRange = 4,     // a member outside [0, n_vertices)
    kErrColOrder = 8,     // a row that is not strictly increasing
    kErrInternal = 16,    // a table probe that found no room (never expected)
    // a replayed batch plan (fixed buffers): the input or the work outgrew it
    kErrPlanShape = 32,   // a graph's row_ptr[0] or row_ptr[m] differs from the plan's
    kErrPlanTasks = 64,   // more counting tasks than the plan's task arrays hold
    kErrPlanPairs = 128,  // more pairs than the plan's result arrays hold
};

// Tunable launch parameters of the counting kernels (the autotuner sets them).
struct Tuning {
    int32_t small_max_wedges = 512;  // items with W_a up to this go to the one-wave kernel
    int32_t task_wedges = 5000;      // wedges per workgroup task (j sub-range of an item)
    int32_t group_parts = 8;         // consecutive tasks of one item run by one workgroup
    int32_t light_len = 12;          // member runs up to this are walked by one lane
    int32_t small_grid_per_cu = 16;  // one-wave workgroups per CU for the small kernel
    int32_t task_grid_per_cu = 4;    // resident workgroups per CU for the task kernel
    int64_t stage_max_bytes = 96ll << 30;  // cap of the staging pool (one counting pass)
    int32_t dense_min_wedges = 4096;  // cut items into dense sub-ranges when each gets this many wedges
    int32_t small_slots = 1024;  // LDS table of the one-wave kernel: 512, 1024 or 2048 home slots
    int32_t task_slots = 8960;   // LDS table of the task kernel: 4480, 8960, 13440 or 17920 home slots
    int32_t tiny_max_wedges = 10;  // one-task items up to this planning cost go one per lane (0: off)
};

// Scan tile: 256 threads x 8 items.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Table sizes (home slots) of the counting kernels are tuning values
// (Tuning::small_slots, Tuning::task_slots), each kernel built for the sizes
// listed there: 8960 home slots + 64 pad = 9024 packed 4-byte slots lets four
// 256-thread task workgroups share a CU, 13440 two; 17920 runs with 512
// threads, two workgroups per CU.
constexpr int kTaskThreads = 256;
// Tiny items (one lane each): at most kTinyCap members and kTinyCap wedges.
// The planning cost is at least a third of the wedges (lookup-only members
// lower it no further), so tiny_max_wedges <= kTinyMaxCost keeps every
// tiny item's wedges within kTinyCap.
constexpr int kTinyCap = 32;
constexpr int kTinyMaxCost = 10;
constexpr int kTinyThreads = 256;

// ------------------------------------------------------------ launchers
// Every launcher enqueues on `st` and returns the launch status.

hipError_t launch_check_rowptr(hipStream_t st, const int32_t *rp, int32_t m, int32_t *err);
hipError_t launch_rows(hipStream_t st, const int32_t *rp, const int32_t *col, int32_t m,
                       int32_t n, int64_t nnz, int check_order, int32_t *rowid, int32_t *err);

hipError_t launch_fill_i32(hipStream_t st, int32_t *p, int64_t n, int32_t v);
hipError_t launch_fill_i64(hipStream_t st, int64_t *p, int64_t n, int64_t v);
hipError_t launch_copy_i32(hipStream_t st, int32_t *dst, const int32_t *src, int64_t n);

// Exclusive scan: out[0..n] with out[n] = total.  `partial` needs
// scan_partials(n) entries of the accumulator type.
int64_t scan_partials(int64_t n);
hipError_t launch_scan_i32(hipStream_t st, const int32_t *in, int64_t n, int32_t *out,
                           int32_t *partial);
hipError_t launch_scan_i32_to_i64(hipStream_t st, const int32_t *in, int64_t n, int64_t *out,
                                  int64_t *partial);

// start[k] = map[k] + 1 (unfiltered member lists)
hipError_t launch_start_from_map(hipStream_t st, int64_t nnz, const int32_t *map, int32_t *start);

// Transpose of an nnz-entry CSR with members in [0, n): ptrT (n + 1), colT
// (the item rowid[k] of each incidence, grouped by member, items ascending),
// kT[q] = the incidence at transposed slot q and posT[k] = its slot (kT,
// posT may be null).  A stable least-significant-digit radix sort of the
// (member, incidence) pairs; rsK / rsV are two pairs of nnz-entry buffers,
// hist holds transpose_hist(nnz) counts and part32 the partials of their
// scan.
int64_t transpose_tiles(int64_t nnz);
int64_t transpose_hist(int64_t nnz);
// Radix passes of a transpose over members in [0, n); its sorted members end
// in rsK[(passes - 1) & 1].
int transpose_passes(int32_t n);
hipError_t launch_transpose(hipStream_t st, const int32_t *col, int64_t nnz, int32_t n,
                            const int32_t *rowid, int32_t *const rsK[2], int32_t *const rsV[2],
                            int32_t *hist, int32_t *part32, int32_t *ptrT, int32_t *colT,
                            int32_t *kT, int32_t *posT);

// s filter: N_s(v) = the items of N(v) with |S| >= s (s_item[it] for item it
// when s_item is given), every list in its order, written to itmS with list
// pointers ptrS (M + 1 entries).  pos (nnz + 1 entries) receives the kept
// entries before each member-list entry; part32 holds the scan's partials.
// With start given, the back-pointer of every kept entry is written as well:
// start[inv[p]] = (its position in itmS) + 1, inv mapping member-list
// positions to item incidences.
// kept (N entries, scratch) receives each item's keep flag first.
hipError_t launch_filter(hipStream_t st, const int32_t *ptrM, const int32_t *itmM, int32_t M,
                         int64_t nnz, const int32_t *ptrI, int32_t N, int32_t s,
                         const int32_t *s_item, int32_t *kept, int32_t *pos, int32_t *part32,
                         int32_t *ptrS, int32_t *itmS, const int32_t *inv, int32_t *start);

// Per-item exact wedge count W_a, the back-pointer start[k] (first item > a
// in N_s(v) for member incidence k of a kept item a) and the run totals:
// totals[0] = kept items, [1] = kept incidences, [2] = wedges.
// full != 0 (product mode): start[k] = the first entry of N_s(v) and W_a counts
// every b in the lists, a itself included.
hipError_t launch_cost(hipStream_t st, const int32_t *ptrI, const int32_t *memI, int32_t N,
                       int32_t s, const int32_t *s_item, const int32_t *ptrS, const int32_t *itmS,
                       int64_t *cost, int32_t *start, int64_t *totals, int32_t full = 0,
                       int32_t have_start = 0);

// Keep the entries (a, b, w) with b > a and w >= s of a row-sorted product,
// in order: pass 1 (out_a == nullptr) counts per block into cnt, pass 2 writes
// at the exclusive scan off of those counts.  kFilterTile entries per block.
constexpr int kFilterTile = 4096;
hipError_t launch_product_filter(hipStream_t st, const int32_t *a, const int32_t *b, const int32_t *w,
                                 int64_t n, int32_t s, int32_t *cnt, const int64_t *off,
                                 int32_t *out_a, int32_t *out_b, int32_t *out_w);

// Lookup-only members (insertion cutoff, s > 1): a candidate b with
// |S_a & S_b| >= s lies in at least s of the lists N_s(v), v in S_a, so if up
// to s - 1 members of a only count candidates that the other members inserted
// before them, every such b is still counted exactly; the others stay below s
// and are dropped.  The longest lists (most wedges) are chosen; the choice is
// flagged in the sign bit of start[k], and cost[a] is lowered to the planning
// cost max(W_a - flagged wedges, W_a / 3).
constexpr int32_t kStartMask = 0x7fffffff;
constexpr int32_t kMaxLookup = 15;  // lookup-only members per item at most
// s_item (nullable) gives each item its own s (batches); s_max is the largest.
// Items with at most kTinyCap members and at most tiny_max wedges (0: none)
// are left as they are: the one-lane path counts every wedge of them.
hipError_t launch_mark_lookup(hipStream_t st, const int32_t *ptrI, const int32_t *memI, int32_t N,
                              int32_t s, const int32_t *s_item, int32_t s_max,
                              const int32_t *ptrS, int32_t *start, int64_t *cost,
                              int32_t tiny_max);

// Tasks: item a with W_a wedges becomes P_a tasks (equal sub-ranges of its
// candidate range); ntask[a] = P_a.  Task t of item a (t = tbase[a] + p) is
// listed in small_tasks, with its item in small_items (W_a <= small_max), or
// in big_tasks; counts[0] / [1]
// receive the list lengths.
hipError_t launch_task_count(hipStream_t st, const int64_t *cost, int32_t N, const Tuning &tu,
                             const int32_t *ptrI, const int32_t *item_end, int32_t full,
                             int32_t *ntask);
// big_tasks receives, per group of up to group_parts consecutive tasks of an
// item, the index of the group's first task; counts[1] = number of groups.
// With `abort` given, the kernel does nothing while *abort != 0.
// Tiny one-task items (Tuning::tiny_max_wedges) go to tiny_tasks /
// tiny_items instead of the small lists; counts[2] receives their number.
hipError_t launch_task_fill(hipStream_t st, const int64_t *cost, int32_t N, const Tuning &tu,
                            const int32_t *ptrI, const int32_t *item_end, int32_t full,
                            const int64_t *tbase, int32_t *task_item, int32_t *task_part,
                            int32_t *small_tasks, int32_t *small_items, int32_t *tiny_tasks,
                            int32_t *tiny_items, int32_t *big_tasks, int32_t *counts,
                            const int32_t *abort = nullptr);

// Counting-kernel modes.
enum : int32_t {
    kModeCount = 0,  // pairs per task only
    kModeFill = 1,   // write (a, b, w) at task_off (only tasks flagged in `need`, if given)
    kModeStage = 2,  // pairs per task, and each extracted range's (b, w) into the pool
};

// One staged range: `n` pairs of task `t` at pool[off], destined for
// task_off[t] + rel.
struct StageRec {
    int64_t off;
    int32_t t, rel, n, pad;
};

struct CountArgs {
    int32_t mode;
    const int32_t *ptrI, *memI;  // item lists
    const int32_t *ptrS, *itmS;  // filtered membership lists
    int32_t N, s;
    const int32_t *s_item;       // per-item s (batches), or null: s for every item
    const int32_t *item_end;     // per item: one past the last item of its graph (batches), or null: N
    int32_t full;                // product mode: every candidate b (both triangles and b = a)
    const int64_t *cost;         // W_a per item
    const int32_t *start;        // back-pointers per item incidence (see launch_cost)
    const int32_t *task_item, *task_part;
    int32_t n_tasks;
    const int32_t *small_tasks, *big_tasks;
    const int32_t *small_items;  // item of each small task
    const int32_t *tiny_tasks, *tiny_items;  // tiny tasks (one lane each) and their items
    const int32_t *task_counts;  // [0] small tasks, [1] task groups, [2] tiny tasks
    int32_t *queue;              // big-task queue head (reset by the launcher)
    int32_t *task_cnt;           // count mode: pairs per task
    const int64_t *task_off;     // fill mode: output offset per task (nullptr = count mode)
    int32_t *out_a, *out_b, *out_w;  // out_w null: weights not written (SLINE_NO_WEIGHTS)
    // stage mode: pool of (b, w) pairs and the range log; tasks that found no
    // room are flagged in need[] (need_count counts them) for a fill pass
    int32_t *pool_b, *pool_w;    // pool_w null: weights not staged
    int64_t pool_cap;
    int64_t pool_chunk;          // pool pairs a workgroup reserves at a time
    unsigned long long *pool_head;
    StageRec *log;
    int32_t log_cap;
    int32_t log_chunk;           // log records a workgroup reserves at a time
    int32_t *log_head;
    int32_t *need;
    int32_t *need_count;
    int64_t *passes;             // [0] table passes; task kernel work: [1] incidences,
                                 // [2] wedges, [3] pairs (count and stage modes)
    int32_t *err;
    Tuning tune;
    int32_t n_cu;
    // batches written straight to per-graph outputs (n_graphs > 0; fill and
    // stage-copy writes only): graph g owns the combined items
    // [g_ibase[g], g_ibase[g + 1]) and the pairs [g_off[g], g_off[g + 1]); its
    // arrays are g_out[g], g_out[G + g] and g_out[2G + g] (null without
    // weights), and both ids are written less g_ibase[g]
    // With g_out null, every pair goes to out_a/out_b/out_w at its combined
    // position, both ids less its graph's g_ibase (g_off unused).
    int32_t n_graphs;
    const int64_t *g_ibase, *g_off;
    int32_t *const *g_out;
    // Replayed plans: while *abort != 0 the counting and copy kernels do
    // nothing (the plan's bounds were exceeded, or its input is malformed).
    const int32_t *abort;
};
// `mid` (may be null) is recorded between the one-wave kernel and the task kernel.
hipError_t launch_count(hipStream_t st, const CountArgs &a, hipEvent_t mid = nullptr);

// ---------------------------------------------------------------- batches
// One graph of a batch (a device array of these drives the batch kernels).
struct BatchGraph {
    const int32_t *rp, *col;  // the caller's CSR
    int32_t m, n;             // edges, vertices
    int32_t dual, s;
    int64_t nnz;              // row_ptr[m]: every row must lie inside [0, nnz)
    int64_t ibase, mbase;     // first combined item id, first combined member id
    int64_t dbase, dzbase;    // dual graphs: first row and first entry in XD
    int64_t vdbase;           // dual graphs: first row of XD^T (vertex rows)
};

hipError_t launch_batch_nnz(hipStream_t st, const BatchGraph *gr, int32_t G, int64_t *nnz,
                            int32_t *err);
// XD = rows of the GD dual graphs (graph dual_ids[q] has rows [dbase[q], dbase[q+1])).
hipError_t launch_batch_concat(hipStream_t st, const BatchGraph *gr, const int32_t *dual_ids,
                               const int64_t *dbase, int32_t GD, int64_t E, int32_t *xcol,
                               int32_t *xrow, int32_t *err);
// Combined items: graph g owns [ibase[g], ibase[g + 1]); ptrT / colT = XD^T.
hipError_t launch_batch_len(hipStream_t st, const BatchGraph *gr, const int64_t *ibase, int32_t G,
                            int64_t NI, const int32_t *ptrT, int32_t *len, int32_t *s_item,
                            int32_t *item_end, int32_t *err);
// Combined member lists: zb (G + 1 entries) receives each graph's first
// combined incidence; memC[ZT] the member ids (one thread per incidence),
// members out of range reported in *err (kErrColRange).  The order of the
// members within a row is left to the row check of the combined lists.
// The concat, length and row kernels do nothing once kErrPlanShape is set in
// *err (a replayed plan then keeps the lists of its previous run).
hipError_t launch_batch_rows(hipStream_t st, const BatchGraph *gr, const int64_t *ibase, int32_t G,
                             int64_t ZT, const int32_t *ptrT, const int32_t *colT,
                             const int32_t *ptrC, int32_t *zb, int32_t *memC, int32_t *err);
hipError_t launch_batch_bounds(hipStream_t st, const int64_t *ibase, int32_t G, const int32_t *a,
                               int64_t P, int64_t *off);
hipError_t launch_batch_split(hipStream_t st, const int64_t *ibase, const int64_t *off, int32_t G,
                              const int32_t *a, const int32_t *b, const int32_t *w, int64_t P,
                              int32_t *const *oa, int32_t *const *ob, int32_t *const *ow);

// g_off[g] = task_off of the first task whose item is >= g_ibase[g], for
// g = 0..G (task_item is non-decreasing; task_off has n_tasks + 1 entries).
// n_tasks_dev (nullable): the task count on the device, read as
// min(*n_tasks_dev, n_tasks) (n_tasks is then the task arrays' capacity).
hipError_t launch_batch_graph_off(hipStream_t st, const int32_t *task_item, int32_t n_tasks,
                                  const int64_t *task_off, const int64_t *g_ibase, int32_t G,
                                  int64_t *g_off, const int64_t *n_tasks_dev = nullptr);

// Replayed plans.  Per graph: row_ptr[0] == 0 and row_ptr[m] == the planned
// nnz, else kErrPlanShape in *err.  And: *value > cap sets `bit` in *err.
hipError_t launch_plan_check_shape(hipStream_t st, const BatchGraph *gr, int32_t G, int32_t *err);
hipError_t launch_plan_guard(hipStream_t st, const int64_t *value, int64_t cap, int32_t bit,
                             int32_t *err);

// Copy staged ranges to their final place (skipping tasks flagged in need).
// n_rec < 0: the records are counted on the device (*log_head, at most
// log_cap), for launches whose sizes are fixed in advance.
hipError_t launch_stage_copy(hipStream_t st, const CountArgs &a, int32_t n_rec);

// ------------------------------------------------- stages (sline_stages.hip)
// Filter of a weighted edge list: pairs with w >= s, in order.  Pass 1
// (oa == nullptr) writes per-tile counts, pass 2 writes at the exclusive scan
// off of those counts.
int64_t wfilter_tiles(int64_t n);
hipError_t launch_wfilter(hipStream_t st, const int32_t *a, const int32_t *b, const int32_t *w,
                          int64_t n, int32_t s, int32_t *cnt, const int64_t *off, int32_t *oa,
                          int32_t *ob, int32_t *ow);
// flag[x] = 1 for items in a pair (flag zeroed by the caller); err gets
// kErrColRange for an id out of [0, N) or a >= b, kErrColOrder for pairs out
// of (a, b) order.
hipError_t launch_mark_present(hipStream_t st, const int32_t *a, const int32_t *b, int64_t n,
                               int32_t N, int32_t *flag, int32_t *err);
hipError_t launch_old_ids(hipStream_t st, const int32_t *flag, const int32_t *newid, int32_t N,
                          int32_t *old_id);
// ptr[x] (x = 0..N) = first pair with a >= x, for pairs sorted by a.
hipError_t launch_run_starts(hipStream_t st, const int32_t *a, int64_t n, int32_t N, int64_t *ptr);
hipError_t launch_degrees(hipStream_t st, const int64_t *fwd, const int32_t *ptrT, int32_t N,
                          int32_t *deg);
hipError_t launch_row_ptr(hipStream_t st, const int32_t *flag, const int32_t *newid,
                          const int64_t *off, int32_t N, int32_t n_nodes, int64_t *row_ptr);
hipError_t launch_adj_fill(hipStream_t st, int32_t N, const int32_t *flag, const int32_t *newid,
                           const int64_t *off, const int32_t *ptrT, const int32_t *colT,
                           const int32_t *kT, const int64_t *fwd, const int32_t *b,
                           const int32_t *w, int32_t *ocol, int32_t *ow);
hipError_t launch_iota(hipStream_t st, int32_t *p, int64_t n);
// comp[x] = smallest item of x's component in the graph of the pairs.
hipError_t launch_components(hipStream_t st, const int32_t *a, const int32_t *b, int64_t n,
                             int32_t N, int32_t *comp);
hipError_t launch_cc_count(hipStream_t st, const int32_t *comp, const int32_t *flag, int32_t N,
                           unsigned long long *count);
hipError_t launch_gather(hipStream_t st, const int32_t *src, const int32_t *idx, int64_t n,
                         int32_t *dst);
hipError_t launch_map_pairs(hipStream_t st, const int32_t *a, const int32_t *b, int64_t n,
                            const int32_t *perm, int32_t *oa, int32_t *ob);
hipError_t launch_sizes(hipStream_t st, const int32_t *ptr, int32_t N, int32_t *size,
                        int32_t *max_size);
hipError_t launch_size_keys(hipStream_t st, const int32_t *size, int32_t N, const int32_t *max_size,
                            int32_t descending, int32_t *key);
hipError_t launch_invert(hipStream_t st, const int32_t *perm, int32_t N, int32_t *inv);
// Rows of (rp, col) in the order perm: nrp (N + 1, len and part32 scratch), ncol.
hipError_t launch_perm_rows(hipStream_t st, const int32_t *rp, const int32_t *col,
                            const int32_t *perm, int32_t N, int32_t *len, int32_t *nrp,
                            int32_t *part32, int32_t *ncol);
hipError_t launch_row_ids(hipStream_t st, const int32_t *rp, int32_t m, int32_t *rowid);
// One set intersection per wedge (the variants without visited skipping):
// count mode (oa == nullptr) writes each item's accepted pairs to cnt, write
// mode appends them from off[a]; inters (nullable) adds the intersections.
hipError_t launch_wedge_intersect(hipStream_t st, const int32_t *ptrI, const int32_t *memI,
                                  const int32_t *ptrS, const int32_t *itmS, const int32_t *start,
                                  int32_t N, int32_t s, int32_t prune, int32_t shortcut,
                                  int32_t *cnt, const int64_t *off, int32_t *oa, int32_t *ob,
                                  int32_t *ow, unsigned long long *inters, int32_t n_cu);

}  // namespace sl
