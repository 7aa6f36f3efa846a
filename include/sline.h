/*
 * libsline -- s-line graphs of hypergraphs on AMD Instinct MI355X (gfx950).
 *
 * The s-line graph L_s(H) (paper, Sec. III): the items of H are its
 * hyperedges e_1..e_m (or, for the dual hypergraph H*, its vertices); two
 * distinct items a, b are adjacent in L_s(H) when their overlap
 * w_ab = |S_a intersect S_b| is at least s, for an integer s >= 1.  L_1(H)
 * is the ordinary line graph.  The paper's method (Sec. IV-B, IV-C) reaches
 * this exact result by walking only pairs that share a member.
 *
 * Every call below is a plain C function taking plain pointers and sizes.
 * Device pointers are HIP device addresses on the context's device; host
 * pointers are ordinary process memory.  All calls are synchronous with
 * respect to the host: when one returns, its device work has finished on the
 * context's stream.  One context must not be used by two host threads at
 * once.  Every function returns an sline_status; 0 is success.  A failed call
 * leaves its output arguments untouched unless stated otherwise, and
 * sline_last_error() then returns a message.
 */
#ifndef SLINE_H
#define SLINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sline_status;
enum {
    SLINE_OK = 0,
    SLINE_EINVAL = -1,    /* malformed input: see sline_build                */
    SLINE_ENOMEM = -2,    /* an allocation failed                            */
    SLINE_ECAPACITY = -3, /* caller buffers too small; n_pairs holds the need */
    SLINE_EDEVICE = -4,   /* a HIP runtime error; message in sline_last_error */
    SLINE_EBUSY = -5      /* result not ready yet (server polling)           */
};

/* Build flags. */
enum {
    SLINE_SKIP_VALIDATE = 1u, /* skip the strictly-increasing row check (range
                                 checks that guard memory always run)       */
    SLINE_PROFILE = 2u,       /* time the stages with HIP events on the
                                 context's stream (see sline_stats)          */
    SLINE_NO_WEIGHTS = 4u,    /* pairs only: the w array is neither needed nor
                                 written (caller buffers may leave w NULL;
                                 library-allocated results have w = NULL).
                                 Saves a third of the output traffic.      */
    /* Relabel-by-degree (Sec. IV-F): sline_build renumbers the items of the
     * side built by size, largest first (DESC) or smallest first (ASC), ties
     * by id, counts on the renumbered hypergraph and maps the result back to
     * the caller's ids -- same output, different work order.  At most one of
     * the two; results of 2^31 pairs or more are refused (SLINE_EINVAL). */
    SLINE_RELABEL_DESC = 8u,
    SLINE_RELABEL_ASC = 16u,
    /* Heuristic ablation (Sec. IV-C; the variants f0..f4 of Table III are
     * f0 = none of these, f1 = NO_VISITED | NO_SHORTCUT, f2 = NO_PRUNE |
     * NO_SHORTCUT, f3 = NO_PRUNE | NO_VISITED, f4 = all three).  They change
     * the work, never the result (results of 2^31 pairs or more are refused
     * with NO_VISITED).
     *   NO_PRUNE     no degree-based pruning: items smaller than s stay in
     *                the member lists and are walked (they cannot reach s)
     *   NO_VISITED   no visited skipping: one set intersection |S_a & S_b|
     *                (two-pointer merge) per wedge (a, v, b) instead of one
     *                counter increment; a pair enters once, from its first
     *                shared member
     *   NO_SHORTCUT  no short-circuit: with NO_VISITED the intersections run
     *                to the end instead of stopping at s; otherwise every
     *                member inserts candidates (no lookup-only members) */
    SLINE_NO_PRUNE = 32u,
    SLINE_NO_VISITED = 64u,
    SLINE_NO_SHORTCUT = 128u
};

typedef struct sline_ctx sline_ctx;

/* Device memory provider.  alloc returns a device pointer of at least `bytes`
 * bytes usable on `stream` (NULL on failure); free releases it.  When no
 * allocator is given the library uses hipMallocAsync / hipFreeAsync on the
 * context's stream. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, size_t bytes, void *stream, void *user);
    void *user;
} sline_allocator;

/* Incidence CSR of H with rows = hyperedges (the transpose of the paper's
 * n x m incidence matrix I of Sec. III, eq. 1).  Device pointers, caller
 * owned, read only, valid until the call returns.
 *   row_ptr[n_edges + 1]: row_ptr[0] = 0, non-decreasing, row_ptr[n_edges] = nnz
 *   col_idx[nnz]: members of hyperedge i are col_idx[row_ptr[i] .. row_ptr[i+1]),
 *                 strictly increasing (a hyperedge is a set), each in
 *                 [0, n_vertices).
 * Empty rows, singleton rows, duplicate rows and isolated vertices are valid
 * (the indexed-family definition of Sec. III). */
typedef struct {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int32_t n_edges;
    int32_t n_vertices;
} sline_csr;

/* An s-line graph as a structure of arrays, sorted by (a, b) ascending, with
 * a < b and w = |S_a intersect S_b| >= s.  Device pointers.
 *   capacity == 0 on input: the library allocates exactly n_pairs entries of
 *                 a, b, w through the context's allocator; release them with
 *                 sline_edges_free.
 *   capacity > 0 on input: a, b, w are caller buffers of `capacity` entries.
 *                 If the result needs more, the call returns SLINE_ECAPACITY
 *                 with n_pairs = the entries needed, writes nothing else, and
 *                 keeps its counting work: an immediate repeat of the same
 *                 call with larger buffers only writes the result (the input
 *                 is not read again: change its contents in between and the
 *                 repeat still gives the first contents' result). */
typedef struct {
    int64_t n_pairs;
    int64_t capacity;
    int32_t *a;
    int32_t *b;
    int32_t *w;
} sline_edges;

/* Work figures of the last build on a context (host struct, filled by
 * sline_last_stats). */
typedef struct {
    int64_t n_items;      /* items of the side built (m, or n for the dual)      */
    int64_t nnz;          /* incidences of H                                      */
    int64_t nnz_kept;     /* incidences of items with |S| >= s                    */
    int64_t n_kept;       /* items with |S| >= s                                  */
    int64_t wedges;       /* W_s: (a, v, b) with a < b, both kept, v shared       */
    int64_t n_pairs;      /* |L_s|                                                */
    int64_t n_small;      /* items counted by the one-wave kernel                 */
    int64_t n_heavy;      /* items counted by the workgroup (multi-pass) kernel   */
    int64_t passes;       /* table passes made by the workgroup kernel            */
    /* stage times in milliseconds, filled when the build had SLINE_PROFILE  */
    double ms_transpose;  /* row checks + transpose (radix sort by member)        */
    double ms_prepare;    /* s filter, per-item wedge counts, buckets             */
    double ms_count;      /* count pass (counting kernels, pairs per item)        */
    double ms_scan;       /* exclusive scan of pairs per item                     */
    double ms_fill;       /* fill pass (counting kernels writing the pairs)       */
    /* the workgroup counting kernel alone (its count or staging pass)        */
    int64_t heavy_nnz;    /* incidences of the items it counted                   */
    int64_t heavy_wedges; /* wedges it walked                                     */
    int64_t heavy_pairs;  /* pairs it produced                                    */
    double ms_tasks;      /* its run time (SLINE_PROFILE)                         */
    /* sline_build_spgemm only                                                */
    int64_t product_nnz;  /* entries of the materialized product H H^T          */
    double ms_product;    /* product time (host clock)                          */
    double ms_filter;     /* filter time (host clock)                           */
    /* SLINE_NO_VISITED builds only                                           */
    int64_t intersections;/* set intersections made (one per wedge)             */
} sline_stats;

/* Launch parameters of the counting stage (they change speed, never the
 * result).  Defaults suit MI355X; sline_set_tuning rejects values outside the
 * stated ranges with SLINE_EINVAL.
 *   small_max_wedges   items with at most this many wedges are counted by one
 *                      wave each (0..512)
 *   task_wedges        wedges per workgroup task, the unit an item's candidate
 *                      range is cut into (64..1048576)
 *   group_parts        consecutive tasks of one item run by one workgroup (1..1024)
 *   light_len          member runs expected to have at most this many entries
 *                      in a task's range are walked by a single lane (0..64;
 *                      default 12)
 *   small_grid_per_cu  resident one-wave workgroups per CU (1..64)
 *   task_grid_per_cu   resident task workgroups per CU (1..16)
 *   stage_max_bytes    cap of the staging pool that lets one counting pass
 *                      produce the result; tasks that do not fit are counted
 *                      again (>= 0; 0 = always two passes)
 *   dense_min_wedges   an item whose candidates give at least this many
 *                      wedges per sub-range narrow enough for direct
 *                      (unhashed) counters is cut into such sub-ranges
 *                      (0..2^24; 0 = sub-ranges by wedge count only)
 *   small_slots        home slots of the one-wave kernel's LDS table: 512,
 *                      1024 or 2048 (small_max_wedges at most half of it)
 *   task_slots         home slots of the task kernel's LDS table: 4480 or 8960
 *                      (256-thread workgroups, four per CU), 13440 (256
 *                      threads, two per CU) or 17920 (512 threads, two per
 *                      CU); larger tables cut fewer sub-ranges per item
 *   tiny_max_wedges    in builds of at least 32768 items, items with a
 *                      planning cost of at most this (and at most 32 members)
 *                      are counted one per lane, by sorting their candidates
 *                      (0..10; 0 = off) */
typedef struct {
    int32_t small_max_wedges;
    int32_t task_wedges;
    int32_t group_parts;
    int32_t light_len;
    int32_t small_grid_per_cu;
    int32_t task_grid_per_cu;
    int64_t stage_max_bytes;
    int32_t dense_min_wedges;
    int32_t small_slots;
    int32_t task_slots;
    int32_t tiny_max_wedges;
} sline_tuning;

/* Create a context on HIP device `device` issuing work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  `alloc` may be NULL; it is
 * copied.  Returns SLINE_EDEVICE if the device cannot be used. */
sline_status sline_create(sline_ctx **ctx, int device, void *hip_stream,
                          const sline_allocator *alloc);

/* Release a context and its workspace.  NULL is allowed. */
void sline_destroy(sline_ctx *ctx);

/* Build L_s(H) (dual = 0: items are hyperedges) or L_s(H*) (dual = 1: items
 * are vertices, S_v = { i : v in e_i }) -- Sec. III; computed by counting,
 * for each kept item a, the shared members of every item b > a reachable
 * through a shared member (Sec. IV-B/IV-C: degree pruning of items with
 * |S| < s, strictly upper triangle, each candidate counted once).
 * Errors: SLINE_EINVAL for s < 1, negative sizes, NULL pointers with
 * non-zero sizes, or (unless SLINE_SKIP_VALIDATE) a CSR that breaks the rules
 * of sline_csr; SLINE_ENOMEM, SLINE_ECAPACITY, SLINE_EDEVICE as above.
 * s larger than every item gives an empty result, not an error. */
sline_status sline_build(sline_ctx *ctx, sline_csr H, int32_t s, int32_t dual,
                         uint32_t flags, sline_edges *out);

/* Size of the device scratch array of sline_build_noalloc (bytes, per
 * device).  The library holds it on every device it runs on until the
 * process ends. */
#define SLINE_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sline_build
 * with caller buffers and no allocation or free of any kind.  Every device
 * buffer of the build (CSR checks, transpose, filtered lists, task arrays,
 * staging pool) is carved from a fixed device array of
 * SLINE_NOALLOC_SCRATCH_BYTES that the library keeps per device; the staging
 * pool takes whatever the rest leaves, and tasks that find no room in it are
 * counted again straight into the caller's arrays.
 *   out    caller buffers only: capacity > 0 and a, b (and w unless
 *          SLINE_NO_WEIGHTS) non-NULL, else SLINE_EINVAL.  On success the
 *          result is exactly sline_build's.  If the result needs more than
 *          `capacity` entries the call returns SLINE_ECAPACITY with n_pairs
 *          set and writes nothing else; a retry counts again (the scratch
 *          keeps no work between calls).
 * Arguments, result and other errors as in sline_build, plus SLINE_ENOMEM
 * (with a message naming the bytes needed) when the build's buffers do not
 * fit the scratch array: about 45 bytes per incidence, 30 per item and 60
 * per counting task, so hypergraphs up to a few 10^5 items and about 10^6
 * incidences fit.  The scratch array is shared by every call on a device:
 * calls on one device that overlap in time (several host threads, or
 * contexts on different streams) race on it and must be serialized by the
 * caller.  Every call clears what it needs zeroed. */
sline_status sline_build_noalloc(sline_ctx *ctx, sline_csr H, int32_t s, int32_t dual,
                                 uint32_t flags, sline_edges *out);

/* ------------------------------------------------ after L_s (Table I)
 * L_s stratifies by s: L_s keeps the pairs of L_1 with w >= s, with the same
 * weights (Sec. III), so L_s is L_s' (s' <= s) filtered.  These calls take an
 * edge list on the device as sline_build returns it: n_pairs >= 0, a, b (and
 * w where stated) device arrays of n_pairs entries. */

/* L_s from a weighted L_s' with s' <= s: the pairs of `in` with w >= s, in
 * their order.  in->w is required (SLINE_EINVAL if NULL with pairs).  `out`
 * and the capacity protocol as in sline_build (flags: SLINE_NO_WEIGHTS drops
 * the output weights); a retry after SLINE_ECAPACITY filters again. */
sline_status sline_filter(sline_ctx *ctx, const sline_edges *in, int32_t s, uint32_t flags,
                          sline_edges *out);

/* An s-sweep: L_s for every s of s_list (n_s entries, each >= 1, any order)
 * of one hypergraph and side.  Only the smallest s is counted (sline_build);
 * every other L_s is filtered from the next smaller one.  outs[i] receives
 * L_{s_list[i]}; every outs[i] must have capacity 0 (library-allocated, free
 * each with sline_edges_free).  flags as in sline_build except
 * SLINE_NO_WEIGHTS (the filters need the weights).  On failure no output is
 * left allocated. */
sline_status sline_build_sweep(sline_ctx *ctx, sline_csr H, int32_t n_s, const int32_t *s_list,
                               int32_t dual, uint32_t flags, sline_edges *outs);

/* The line graph as a graph (Sec. IV-E).  Nodes are the items that occur in
 * L, renumbered 0..n_nodes-1 in the order of their ids ("ID squeezing");
 * old_id maps back.  The adjacency is symmetric: pair (a, b, w) is the arc
 * (a', b') in row a' and the arc (b', a') in row b'; every row ascending.
 * All arrays are device memory allocated through the context's allocator;
 * release them with sline_graph_free. */
typedef struct {
    int32_t n_nodes;
    int64_t n_arcs;    /* 2 * n_pairs                                       */
    int32_t *old_id;   /* [n_nodes] original id of each node, ascending     */
    int64_t *row_ptr;  /* [n_nodes + 1]                                     */
    int32_t *col;      /* [n_arcs] neighbours (squeezed ids)                */
    int32_t *w;        /* [n_arcs] overlaps, NULL with SLINE_NO_WEIGHTS     */
} sline_graph;

/* Squeeze L (pairs of items in [0, n_items), sorted by (a, b), a < b) and
 * build its adjacency (Sec. IV-E).  L->w is required unless flags has
 * SLINE_NO_WEIGHTS.  SLINE_EINVAL for ids out of range, pairs out of order or
 * n_pairs >= 2^31; SLINE_ENOMEM, SLINE_EDEVICE as usual.  On failure *G is
 * left untouched. */
sline_status sline_squeeze(sline_ctx *ctx, int32_t n_items, const sline_edges *L, uint32_t flags,
                           sline_graph *G);

/* Release the arrays of a graph from sline_squeeze and zero the struct. */
sline_status sline_graph_free(sline_ctx *ctx, sline_graph *G);

/* s-connected components (Table I): the connected components of the graph
 * L on items 0..n_items-1 (L as in sline_squeeze, weights not read).
 *   comp          device int32[n_items], caller-owned: comp[x] = the
 *                 smallest item of x's component (an item in no pair is its
 *                 own component)
 *   n_components  host, may be NULL: components with at least two items
 *                 (those of the squeezed graph)
 * Errors as in sline_squeeze (any n_pairs is accepted). */
sline_status sline_components(sline_ctx *ctx, int32_t n_items, const sline_edges *L,
                              int32_t *comp, int64_t *n_components);

/* Companion route to the same result (Sec. IV-D): the product C = H H^T
 * (H* H*^T for dual = 1) with both triangles and the diagonal, computed row
 * by row (Gustavson) with the LDS hash accumulators of sline_build and
 * materialized in full -- nnz(C) = 2 |L_1| + (non-empty items) entries of 12
 * bytes -- then filtered to the pairs with b > a and w >= s.  No degree
 * pruning: the product does not depend on s.  Arguments, output, errors and
 * the capacity protocol as in sline_build (SLINE_ECAPACITY computes the
 * product again on the retry).  Built for comparison with sline_build. */
sline_status sline_build_spgemm(sline_ctx *ctx, sline_csr H, int32_t s, int32_t dual,
                                uint32_t flags, sline_edges *out);

/* Build L_{s[g]} of every hypergraph Hs[g] (dual[g] as in sline_build) in
 * one pass of the counting pipeline: the graphs' items are numbered one after
 * the other, every item is compared against its own graph's s, and the pairs
 * are split back per graph (the result of graph g is exactly what
 * sline_build(ctx, Hs[g], s[g], dual[g], ...) returns).  The method is that of
 * sline_build (Sec. IV-B/IV-C); batching only changes how many launches a
 * set of graphs costs.
 *   n_graphs   >= 0 (0: nothing to do)
 *   Hs, s, dual, outs   host arrays of n_graphs entries; the CSR arrays they
 *              point at are device memory owned by the caller
 *   outs[g]    as in sline_build: capacity 0 lets the library allocate graph
 *              g's arrays (free each with sline_edges_free); capacity > 0
 *              supplies caller buffers.  If any graph's buffers are too small
 *              the call returns SLINE_ECAPACITY, sets n_pairs of every graph
 *              and writes no pairs; an immediate retry with the same
 *              arguments (larger buffers) reuses the computed result (the
 *              graphs are not read again).
 * Errors: SLINE_EINVAL if any graph is malformed (as in sline_build) or any
 * s[g] < 1 / dual[g] not in {0, 1}; the combined item and member counts and
 * incidences must each stay below 2^31.  Other codes as above. */
sline_status sline_build_batch(sline_ctx *ctx, int32_t n_graphs, const sline_csr *Hs,
                               const int32_t *s, const int32_t *dual, uint32_t flags,
                               sline_edges *outs);

/* ---------------------------------------------------------- batch plans
 * A batch (as in sline_build_batch) sized once and then replayed as one HIP
 * graph launch: no size read-back and no allocation between its ~40 kernels,
 * one read-back of the per-graph pair counts at the end.  Not a step of the
 * paper: it is the launch form of repeated batched builds (the same graphs,
 * rebuilt after their member lists change in place, or swept to larger s).
 *
 * sline_batch_plan_create checks the graphs, runs the batch's counting once
 * to learn its sizes, then allocates every buffer of the pipeline through the
 * context's allocator -- the combined item lists, the transposes, the task
 * arrays (exactly the tasks counted), the staging pool (W_s / s_min pairs,
 * capped by the tuning's stage_max_bytes) and the result arrays (exactly the
 * pairs counted) -- and captures the pipeline on a stream of its own into a
 * graph.  It uses the context's tuning as it is at creation.  The graphs'
 * arrays are the caller's: they must stay allocated, with the same row_ptr[m],
 * n_edges and n_vertices, for the plan's lifetime; their contents may change
 * between runs.
 *
 * sline_batch_plan_run launches the graph on the context's stream and waits
 * for it.  s (nullable: the planned values) gives each graph's s for this
 * run; each must be >= the planned s of its graph (larger s only shrinks the
 * work and the result, Sec. III).  outs[g] receives graph g's L_s in the
 * plan's own result arrays: a, b, w (w null with SLINE_NO_WEIGHTS) point into
 * them, n_pairs is set and capacity is 0.  They stay valid until the next run
 * or sline_batch_plan_destroy; never pass them to sline_edges_free.
 * Results equal sline_build_batch's for the same graphs, s and flags.
 * Errors (outs untouched unless SLINE_OK):
 *   SLINE_EINVAL     bad arguments; a graph breaks the rules of sline_csr, or
 *                    its row_ptr[0] / row_ptr[m] changed since the plan was made;
 *                    a run's s below the planned s (checked before anything
 *                    runs: the run changes nothing); flags other than
 *                    SLINE_NO_WEIGHTS.
 *   SLINE_ECAPACITY  the run needs more tasks or pairs than the plan holds
 *                    (changed contents); make a new plan.
 *   SLINE_ENOMEM     allocation failed (create only).
 *   SLINE_EDEVICE    a HIP call failed (graph capture included).
 * A plan belongs to its context: use it from one thread at a time with the
 * context's other calls, and destroy it before the context. */
typedef struct sline_batch_plan sline_batch_plan;

sline_status sline_batch_plan_create(sline_ctx *ctx, int32_t n_graphs, const sline_csr *Hs,
                                     const int32_t *s, const int32_t *dual, uint32_t flags,
                                     sline_batch_plan **plan);
sline_status sline_batch_plan_run(sline_batch_plan *plan, const int32_t *s, sline_edges *outs);
/* Device bytes the plan holds, and its task and pair capacities. */
sline_status sline_batch_plan_info(const sline_batch_plan *plan, int64_t *device_bytes,
                                   int64_t *task_capacity, int64_t *pair_capacity);
void sline_batch_plan_destroy(sline_batch_plan *plan);

/* ------------------------------------------------------------- serving
 * A query loop over resident hypergraphs.  Registered graphs stay where the
 * caller keeps them (device CSR arrays that must outlive the server).
 * Queries (graph, s, side) are queued on submit; each of the server's worker
 * threads owns a context on its own HIP stream and, whenever idle, takes the
 * queued queries in arrival order that fit the device-memory budget next to
 * the batches already running, and counts them as one batched build
 * (sline_build_batch).  Queries arriving meanwhile join the next batch, so
 * batches of different workers overlap on the device.  A query's result is
 * exactly the plain build of its graph, s and side.  The workers' device
 * memory comes from the server's own allocator: chunks of at least 4 GiB from
 * hipMalloc, carved by best fit and kept until the server is destroyed (chunks
 * with nothing allocated are returned when hipMalloc fails).  Setting the
 * environment variable SLINE_SERVER_LOG prints one line per batch to stderr. */
typedef struct sline_server sline_server;

/* Timing and outcome of one query (host steady clock, nanoseconds). */
typedef struct {
    int64_t n_pairs;
    int64_t t_submit_ns;  /* sline_server_submit                            */
    int64_t t_start_ns;   /* its batch was taken by a worker                 */
    int64_t t_done_ns;    /* result complete on the device                   */
    int32_t batch_size;   /* queries counted in the same batched build       */
    int32_t status;       /* sline_status of the query                       */
} sline_query_info;

/* Start a server on `device` with `n_workers` (1..16) worker threads.
 * hbm_budget_bytes caps the estimated device memory of the batches running
 * at once plus the results handed over and not yet released (a single query
 * above the cap still runs, alone, when nothing else runs); max_batch caps
 * the queries per batch.  The estimate of a query is about 80 bytes per
 * incidence plus 20 bytes per pair the result can hold (W_1 / s, where W_1 is
 * the sum over members of C(degree, 2) on the query's side, at most
 * N(N - 1) / 2).  The server reserves the budget as device memory when it
 * starts (if the device has it to spare) and holds its memory until
 * sline_server_destroy; beyond the reservation it grows only while a
 * sixteenth of the device (at least 16 GiB) stays free. */
sline_status sline_server_create(sline_server **srv, int device, int64_t hbm_budget_bytes,
                                 int32_t max_batch, int32_t n_workers);

/* Register a hypergraph (device CSR as in sline_build, caller-owned) and get
 * its id.  Reads the CSR once to size queries and checks it against the rules
 * of sline_csr (row_ptr[0] = 0, row_ptr non-decreasing, members
 * in range and strictly increasing within a row): SLINE_EINVAL if it breaks
 * one, so a malformed graph never joins a batch.  (A batch that still fails
 * with SLINE_EINVAL or SLINE_ENOMEM is run again one query at a time, so
 * every query gets the status of its own plain build.) */
sline_status sline_server_register(sline_server *srv, sline_csr H, int32_t *graph_id);

/* Queue the query L_s of graph `graph_id` (dual as in sline_build). */
sline_status sline_server_submit(sline_server *srv, int32_t graph_id, int32_t s, int32_t dual,
                                 int64_t *ticket);

/* SLINE_EBUSY while the query is queued or running.  Otherwise the ticket is
 * retired: `info` (may be NULL) receives its timing, and on SLINE_OK `out`
 * receives the result arrays (device memory owned by the server until
 * sline_server_release; out->capacity is 0).  A query that failed returns its
 * status; sline_server_last_error has the message.  Unknown tickets give
 * SLINE_EINVAL. */
sline_status sline_server_poll(sline_server *srv, int64_t ticket, sline_edges *out,
                               sline_query_info *info);

/* Free a result handed over by sline_server_poll, once no device work reads
 * it any more, and zero the struct. */
sline_status sline_server_release(sline_server *srv, sline_edges *out);

/* Result reuse.  L_s keeps the pairs of L_s' (s' <= s) with w >= s, with
 * the same weights (Sec. III).  The server keeps, per (graph, side), a copy
 * of the result of the smallest s computed so far, for graphs of at least
 * min_nnz incidences, within cache_bytes of device memory beside the
 * budget (one result at most half of it; least recently used first out; a
 * build that runs out of device memory drops them and is tried again).  A later query of
 * that graph and side with s >= the kept s is answered by sline_filter from
 * it instead of a build; the answer is the same.  cache_bytes = 0 turns
 * reuse off and drops what is kept.  Defaults: a quarter of the budget (at
 * most 32 GiB), min_nnz = 2^20, no flags.
 * flags: SLINE_REUSE_LOOKAHEAD -- a query of s > 2 that must build looks at
 * the queued queries of its graph and side and builds at the smallest s
 * (>= 2) among them; its own answer is that build filtered to its s, and the
 * others wait for the build and are answered from the kept result.  Queued
 * queries that a kept result answers are then admitted before the others
 * (each is one filter), while their result is still kept.  It pays when
 * cache_bytes holds a result for the graphs and sides in use; with less, the
 * larger builds are evicted before they are reused. */
#define SLINE_REUSE_LOOKAHEAD 1u
sline_status sline_server_set_reuse(sline_server *srv, int64_t cache_bytes, int64_t min_nnz,
                                    uint32_t flags);

/* Queries answered by reuse, results kept so far, and bytes kept now (any
 * pointer may be NULL). */
sline_status sline_server_reuse_stats(sline_server *srv, int64_t *reused, int64_t *kept,
                                      int64_t *kept_bytes);

/* Queries waiting and batches running (either pointer may be NULL). */
sline_status sline_server_pending(sline_server *srv, int64_t *queued, int32_t *running);

/* Message of the last failed batch ("" if none). */
const char *sline_server_last_error(sline_server *srv);

/* Stop the workers (queries still queued are dropped), free every result not
 * yet released and the server.  NULL is allowed. */
void sline_server_destroy(sline_server *srv);

/* Release the arrays of a library-allocated result and zero the struct.
 * Caller-owned buffers (capacity > 0) are not touched. */
sline_status sline_edges_free(sline_ctx *ctx, sline_edges *edges);

/* Read / replace the context's launch parameters (host structs). */
sline_status sline_get_tuning(sline_ctx *ctx, sline_tuning *tuning);
sline_status sline_set_tuning(sline_ctx *ctx, const sline_tuning *tuning);

/* Statistics of the last successful build on `ctx`. */
sline_status sline_last_stats(sline_ctx *ctx, sline_stats *stats);

/* Static text for a status code. */
const char *sline_status_str(sline_status status);

/* Message of the last failed call on `ctx` ("" if none); valid until the next
 * call on the context.  Includes the HIP error text for SLINE_EDEVICE. */
const char *sline_last_error(sline_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SLINE_H */
