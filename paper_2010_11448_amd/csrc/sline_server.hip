// Serving: a query loop over resident hypergraphs with continuous batching.
//
// Queries (graph, s, side) arrive at any time.  Each worker thread owns a
// library context on its own HIP stream; whenever it is idle it takes, in
// arrival order, the queued queries that fit the device-memory budget next
// to the work already in flight, and runs them as one batched build.  Queries
// that arrive while a batch runs are taken by the next idle worker, so
// batches of different workers overlap on the device.  A query's result is
// exactly that of a plain build of the same graph, s and side: batching only
// shares launches between independent graphs.
//
// Admission estimate of a query (bytes): the pipeline's workspace, about
// 80 bytes per incidence, plus 20 bytes per possible pair, where the pairs of
// L_s are bounded by W_1 / s (every pair of L_s takes at least s of the W_1
// wedges of its side, W_1 = sum over members of C(degree, 2)) and by
// N(N - 1) / 2.  W_1 of both sides is computed when a graph is registered.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sline.h"
#include "sline_internal.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Graph {
    sline_csr H{};
    int64_t nnz = 0;
    double w1[2] = {0, 0};  // W_1 of the primal and the dual side
};

// Device memory of the workers (and of handed-over results): large chunks
// from hipMalloc, carved into blocks by best fit and merged again on release,
// so the serving loop maps device memory once instead of per query (mapping
// fresh memory costs more than most builds).  The budget is reserved as one
// chunk when the server starts.  A further chunk is only requested while the
// device keeps a sixteenth of its memory (at least 16 GiB) free: near a full
// device, hipMalloc calls were measured at seconds each, failing or not,
// and no worker could allocate meanwhile.  (The budget itself is kept by
// admission, which lets a query larger than the budget run alone.)  When no
// chunk has room, chunks with nothing allocated are returned first; if that
// does not make room the request fails at once and the library takes its
// fallback (a smaller staging pool, or an error the worker answers by
// running the batch's queries apart).
struct DeviceCache {
    struct Chunk {
        char *base = nullptr;
        size_t size = 0, used = 0;
        std::map<size_t, size_t> free;  // offset -> length, merged
    };
    std::mutex mu;
    std::vector<Chunk *> chunks;
    std::map<void *, std::pair<Chunk *, size_t>> live;  // block -> (chunk, length)
    size_t chunk_min = (size_t)4 << 30;
    size_t total = 0;                           // bytes the chunks add up to
    // device calls made so far (reported by the server log)
    int64_t n_malloc = 0, n_malloc_fail = 0, n_free = 0, ns_malloc = 0, ns_free = 0;

    static size_t round(size_t n) {
        const size_t g = (size_t)2 << 20;
        return (std::max<size_t>(n, 1) + g - 1) & ~(g - 1);
    }

    // best fit over all chunks; caller holds mu
    void *carve(size_t n) {
        Chunk *bc = nullptr;
        size_t boff = 0, blen = SIZE_MAX;
        for (Chunk *c : chunks)
            for (auto &f : c->free)
                if (f.second >= n && f.second < blen) {
                    bc = c;
                    boff = f.first;
                    blen = f.second;
                }
        if (!bc) return nullptr;
        bc->free.erase(boff);
        if (blen > n) bc->free[boff + n] = blen - n;
        bc->used += n;
        void *p = bc->base + boff;
        live[p] = {bc, n};
        return p;
    }

    // device memory a new chunk may take: what is free beyond the headroom
    static size_t growable() {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        const size_t headroom = std::max((size_t)16 << 30, tot / 16);
        return fr > headroom ? fr - headroom : 0;
    }

    // bytes a new chunk for a request of n bytes may have (0: none)
    size_t grow_size(size_t n) const {
        const size_t avail = growable();
        if (n > avail) return 0;
        return std::min(std::max(n, chunk_min), avail);
    }

    // one chunk of up to `bytes` (less if the device has less to spare)
    void reserve(size_t bytes) {
        std::lock_guard<std::mutex> lk(mu);
        const size_t sz = round(std::min(bytes, growable()));
        if (sz < chunk_min) return;
        void *base = nullptr;
        if (hipMalloc(&base, sz) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        Chunk *c = new Chunk();
        c->base = static_cast<char *>(base);
        c->size = sz;
        c->free[0] = sz;
        chunks.push_back(c);
        total += sz;
    }

    void *alloc(size_t n) {
        n = round(n);
        std::lock_guard<std::mutex> lk(mu);
        if (void *p = carve(n)) return p;
        for (int attempt = 0; attempt < 2; ++attempt) {
            const size_t sz = grow_size(n);
            if (sz == 0) {
                if (attempt == 0 && release_empty()) continue;
                return nullptr;
            }
            void *base = nullptr;
            const int64_t t0 = now_ns();
            const hipError_t e = hipMalloc(&base, sz);
            ns_malloc += now_ns() - t0;
            ++n_malloc;
            if (e == hipSuccess) {
                Chunk *c = new Chunk();
                c->base = static_cast<char *>(base);
                c->size = sz;
                c->free[0] = sz;
                chunks.push_back(c);
                total += sz;
                return carve(n);
            }
            (void)hipGetLastError();
            ++n_malloc_fail;
            if (attempt == 0) release_empty();
        }
        return nullptr;
    }

    void release(void *p, hipStream_t st) {
        if (!p) return;
        // the block may next serve another stream: let this one finish with it
        if (st) (void)hipStreamSynchronize(st);
        std::lock_guard<std::mutex> lk(mu);
        auto it = live.find(p);
        if (it == live.end()) return;
        Chunk *c = it->second.first;
        size_t off = static_cast<char *>(p) - c->base, len = it->second.second;
        live.erase(it);
        c->used -= len;
        auto nx = c->free.lower_bound(off);
        if (nx != c->free.end() && off + len == nx->first) {
            len += nx->second;
            nx = c->free.erase(nx);
        }
        if (nx != c->free.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        c->free[off] = len;
    }

    // caller holds mu; returns whether a chunk was freed
    bool release_empty() {
        std::vector<Chunk *> keep;
        bool freed = false;
        for (Chunk *c : chunks) {
            if (c->used == 0) {
                freed = true;
                total -= c->size;
                const int64_t t0 = now_ns();
                (void)hipFree(c->base);
                ns_free += now_ns() - t0;
                ++n_free;
                delete c;
            } else {
                keep.push_back(c);
            }
        }
        chunks.swap(keep);
        return freed;
    }

    void destroy() {
        std::lock_guard<std::mutex> lk(mu);
        for (Chunk *c : chunks) {
            (void)hipFree(c->base);
            delete c;
        }
        chunks.clear();
        live.clear();
        total = 0;
    }
};

void *cache_alloc(size_t n, void *stream, void *user) {
    (void)stream;
    return static_cast<DeviceCache *>(user)->alloc(n);
}

void cache_free(void *p, size_t n, void *stream, void *user) {
    (void)n;
    static_cast<DeviceCache *>(user)->release(p, static_cast<hipStream_t>(stream));
}

struct Query {
    int64_t ticket = 0;
    int32_t graph = 0, s = 1, dual = 0;
    int32_t s_build = 1;  // s its build runs at (<= s; below s, filtered to s after)
    int64_t est = 0;
    bool reused = false;  // answered by filtering a kept result
    sline_query_info info{};
    sline_edges out{};
    bool done = false;
    int32_t worker = -1;
};

}  // namespace

struct sline_server {
    int device = 0;
    int64_t budget = 0;
    int32_t max_batch = 64;
    std::vector<Graph> graphs;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int64_t> queue;                    // tickets waiting, in arrival order
    std::unordered_map<int64_t, Query> queries;   // every ticket not yet handed over
    int64_t next_ticket = 1;
    int64_t in_flight = 0;                        // estimated bytes of running batches
    int64_t held = 0;                             // bytes of results not yet released
    int32_t running = 0;                          // batches on the device
    bool stop = false;
    struct Worker {
        sline_ctx *ctx = nullptr;
        hipStream_t stream = nullptr;
        std::thread th;
    };
    std::vector<Worker> workers;
    DeviceCache cache;                            // device memory of every worker
    bool log = false;                             // SLINE_SERVER_LOG set: one line per batch
    std::string last_error;
    // Result reuse.  L_s keeps the pairs of L_s' (s' <= s) with w >= s, with
    // the same weights (Sec. III), so a kept L_s' answers every later query
    // of the same graph and side with s >= s' by a filter instead of a
    // build.  Per (graph, side) the result of the smallest s computed so far
    // is kept (a copy in the device cache), within reuse_cap bytes, least
    // recently used first out; an entry being filtered from is never freed.
    struct Kept {
        int32_t s = 0;
        sline_edges e{};
        int64_t bytes = 0;
        int64_t last = 0;
        int32_t users = 0;
    };
    std::map<std::pair<int32_t, int32_t>, Kept> kept;
    // result arrays shared by a client and a kept entry: owners beyond one
    std::unordered_map<void *, int32_t> extra_refs;
    // (graph, side) being built by a running batch: the smallest s; a query
    // of the same key with s at least that waits for the result to be kept
    std::map<std::pair<int32_t, int32_t>, int32_t> building;
    int64_t kept_bytes = 0;
    int64_t reuse_cap = 0;      // bytes the kept results may hold (0: no reuse)
    int64_t reuse_min_nnz = 0;  // graphs with fewer incidences are not kept
    bool lookahead = false;     // SLINE_REUSE_LOOKAHEAD
    int64_t use_clock = 0;
    int64_t n_reused = 0, n_kept = 0;  // queries answered by a filter, results kept
};

namespace {

// Device bytes a handed-over result holds until it is released.
int64_t result_bytes(const sline_edges &e) {
    return (int64_t)sizeof(int32_t) * e.n_pairs * (e.w ? 3 : 2);
}

int64_t kept_result_bytes(const sline_edges &e) {
    return (int64_t)sizeof(int32_t) * e.n_pairs * 3;
}

// One owner of a result array lets go (caller holds S->mu): the array is
// freed with its last owner.
void unref(sline_server *S, void *p) {
    if (!p) return;
    auto it = S->extra_refs.find(p);
    if (it != S->extra_refs.end()) {
        if (--it->second > 0) return;
        S->extra_refs.erase(it);
        return;
    }
    S->cache.release(p, nullptr);
}

void add_ref(sline_server *S, void *p) {
    if (p) S->extra_refs[p] += 1;
}

// Let go of the arrays of a kept result (caller holds S->mu; the entry has
// no users).
void drop_kept(sline_server *S, sline_server::Kept &k) {
    unref(S, k.e.a);
    unref(S, k.e.b);
    unref(S, k.e.w);
    S->kept_bytes -= k.bytes;
    k = sline_server::Kept{};
}

// Least recently used kept results out until they fit `cap` (caller holds
// S->mu); entries in use stay.
void evict_kept(sline_server *S, int64_t cap) {
    while (S->kept_bytes > cap) {
        auto victim = S->kept.end();
        for (auto it = S->kept.begin(); it != S->kept.end(); ++it)
            if (it->second.users == 0 && (victim == S->kept.end() || it->second.last < victim->second.last))
                victim = it;
        if (victim == S->kept.end()) return;
        drop_kept(S, victim->second);
        S->kept.erase(victim);
    }
}

// Keep a computed result (its arrays shared with the client, no copy) if it
// is the smallest s of its graph and side so far and fits the reuse budget
// (caller holds S->mu).
void keep_result(sline_server *S, int32_t graph, int32_t dual, int32_t s, const sline_edges &res) {
    const int64_t bytes = kept_result_bytes(res);
    if (S->reuse_cap <= 0 || bytes > S->reuse_cap / 2 || !res.w || res.n_pairs == 0 ||
        S->graphs[graph].nnz < S->reuse_min_nnz)
        return;
    auto it = S->kept.find({graph, dual});
    if (it != S->kept.end()) {
        if (it->second.s <= s || it->second.users > 0) return;
        drop_kept(S, it->second);
    }
    sline_server::Kept &k = S->kept[{graph, dual}];
    k.s = s;
    k.e = sline_edges{res.n_pairs, 0, res.a, res.b, res.w};
    k.bytes = bytes;
    k.last = ++S->use_clock;
    k.users = 0;
    add_ref(S, res.a);
    add_ref(S, res.b);
    add_ref(S, res.w);
    S->kept_bytes += bytes;
    S->n_kept += 1;
    evict_kept(S, S->reuse_cap);
}

int64_t estimate(const Graph &g, int32_t s, int32_t dual) {
    const double N = dual ? g.H.n_vertices : g.H.n_edges;
    const double pairs = std::min(g.w1[dual] / std::max(s, 1), N * (N - 1.0) / 2.0);
    return (int64_t)(80.0 * (double)g.nnz + 20.0 * pairs) + (1 << 20);
}

void free_arrays(sline_server *S, const sline_edges &e);

void worker_loop(sline_server *S, int wi) {
    sline_server::Worker &W = S->workers[wi];
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<int64_t> batch;   // queries counted by one batched build
        std::vector<int64_t> reuse;   // queries filtered from a kept result
        std::vector<sline_edges> from;
        std::vector<std::pair<int32_t, int32_t>> from_key;
        int64_t est = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop) return;
                // queries a kept result answers go first, wherever they are
                // in the queue: each is one filter, and answering them while
                // their result is kept spares a rebuild once it is evicted
                if (S->lookahead && !S->kept.empty()) {
                    for (auto qi = S->queue.begin();
                         qi != S->queue.end() && (int32_t)reuse.size() < S->max_batch;) {
                        Query &q = S->queries[*qi];
                        const std::pair<int32_t, int32_t> key{q.graph, q.dual};
                        auto kt = S->kept.find(key);
                        if (kt == S->kept.end() || kt->second.s > q.s) {
                            ++qi;
                            continue;
                        }
                        const int64_t qe = kt->second.bytes + ((int64_t)1 << 20);
                        const bool alone = S->in_flight == 0 && reuse.empty();
                        if (!alone && S->in_flight + S->held + est + qe > S->budget) break;
                        est += qe;
                        kt->second.users += 1;
                        kt->second.last = ++S->use_clock;
                        q.reused = true;
                        reuse.push_back(q.ticket);
                        from.push_back(kt->second.e);
                        from_key.push_back(kt->first);
                        qi = S->queue.erase(qi);
                    }
                    if (!reuse.empty()) break;
                }
                // admit in arrival order while the batch and the budget allow;
                // a query larger than the budget runs alone when nothing else does
                for (auto qi = S->queue.begin();
                     qi != S->queue.end() && (int32_t)(batch.size() + reuse.size()) < S->max_batch;) {
                    Query &q = S->queries[*qi];
                    const std::pair<int32_t, int32_t> key{q.graph, q.dual};
                    auto kt = S->kept.find(key);
                    const bool can_reuse = kt != S->kept.end() && kt->second.s <= q.s;
                    if (!can_reuse && S->reuse_cap > 0) {
                        // a running build of the same graph and side with a
                        // smaller s will answer this query once it is kept
                        auto bt = S->building.find(key);
                        if (bt != S->building.end() && bt->second <= q.s) {
                            ++qi;
                            continue;
                        }
                    }
                    // Queued queries of the same graph and side that a kept
                    // result could answer: one build at the smallest s (>= 2)
                    // among them answers them all -- this one by a filter of
                    // the build, the others from the kept result -- where
                    // each would otherwise build in turn.
                    int32_t s_build = q.s;
                    if (S->lookahead && !can_reuse && S->reuse_cap > 0 && q.s > 2 &&
                        S->graphs[q.graph].nnz >= S->reuse_min_nnz) {
                        for (const int64_t t2 : S->queue) {
                            const Query &o = S->queries[t2];
                            if (o.graph == q.graph && o.dual == q.dual && o.s >= 2 && o.s < s_build)
                                s_build = o.s;
                        }
                    }
                    // a filtered result is at most the kept one
                    const int64_t qe =
                        can_reuse ? kt->second.bytes + ((int64_t)1 << 20)
                        : s_build == q.s ? q.est
                                         : estimate(S->graphs[q.graph], s_build, q.dual);
                    // results the client has not released count against the
                    // budget too (so a slow client holds back admission); kept
                    // results live beside the budget, within their own cap,
                    // and give way when a build runs out of device memory
                    const bool alone = S->in_flight == 0 && batch.empty() && reuse.empty();
                    const bool fits = S->in_flight + S->held + est + qe <= S->budget;
                    if (!alone && !fits) break;
                    // a build above the whole budget runs alone; kept results
                    // stay unless it runs out of device memory (then they go
                    // and it is tried again)
                    est += qe;
                    if (can_reuse) {
                        kt->second.users += 1;
                        kt->second.last = ++S->use_clock;
                        q.reused = true;
                        reuse.push_back(q.ticket);
                        from.push_back(kt->second.e);
                        from_key.push_back(kt->first);
                    } else {
                        q.s_build = s_build;
                        batch.push_back(q.ticket);
                        auto bt = S->building.find(key);
                        if (bt == S->building.end() || bt->second > s_build) S->building[key] = s_build;
                    }
                    qi = S->queue.erase(qi);
                }
                if (!batch.empty() || !reuse.empty()) break;
                S->cv.wait(lk);
            }
            S->in_flight += est;
            S->running += 1;
        }
        const int32_t G = (int32_t)batch.size();
        const int32_t R = (int32_t)reuse.size();
        std::vector<sline_csr> Hs(G);
        std::vector<int32_t> ss(G), ds(G), gs(G), want(G), rs(R);
        std::vector<sline_edges> outs(G), routs(R);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const int64_t t = now_ns();
            for (int32_t g = 0; g < G; ++g) {
                Query &q = S->queries[batch[g]];
                Hs[g] = S->graphs[q.graph].H;
                ss[g] = q.s_build;
                want[g] = q.s;
                ds[g] = q.dual;
                gs[g] = q.graph;
                outs[g] = sline_edges{};
                q.info.t_start_ns = t;
                q.info.batch_size = G;
                q.worker = wi;
            }
            for (int32_t r = 0; r < R; ++r) {
                Query &q = S->queries[reuse[r]];
                rs[r] = q.s;
                routs[r] = sline_edges{};
                q.info.t_start_ns = t;
                q.info.batch_size = 1;
                q.worker = wi;
            }
        }
        // queries answered from kept results: one filter each
        std::vector<sline_status> rst(R, SLINE_OK);
        for (int32_t r = 0; r < R; ++r) rst[r] = sline_filter(W.ctx, &from[r], rs[r], 0, &routs[r]);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (int32_t r = 0; r < R; ++r) {
                auto kt = S->kept.find(from_key[r]);
                if (kt != S->kept.end()) kt->second.users -= 1;
            }
            S->n_reused += R;
        }
        std::string rerr;
        for (int32_t r = 0; r < R; ++r)
            if (rst[r] != SLINE_OK) rerr = sline_last_error(W.ctx);
        int64_t c0[5] = {0, 0, 0, 0, 0};
        if (S->log) {
            std::lock_guard<std::mutex> lk(S->cache.mu);
            c0[0] = S->cache.n_malloc;
            c0[1] = S->cache.n_malloc_fail;
            c0[2] = S->cache.n_free;
            c0[3] = S->cache.ns_malloc;
            c0[4] = S->cache.ns_free;
        }
        const int64_t t_run = now_ns();
        const uint32_t flags = S->log ? SLINE_PROFILE : 0;
        sline_status st = G > 0 ? sline_build_batch(W.ctx, G, Hs.data(), ss.data(), ds.data(), flags,
                                                    outs.data())
                                : SLINE_OK;
        if (st == SLINE_ENOMEM) {
            // kept results give way to builds: drop those not being read, retry
            bool dropped = false;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                const int64_t before = S->kept_bytes;
                evict_kept(S, 0);
                dropped = S->kept_bytes < before;
            }
            if (dropped) {
                for (auto &o : outs) o = sline_edges{};
                st = sline_build_batch(W.ctx, G, Hs.data(), ss.data(), ds.data(), flags, outs.data());
            }
        }
        // per query: the batch's status, or its own when the batch ran apart
        std::vector<sline_status> qst(G, st);
        const bool apart = (st == SLINE_ENOMEM || st == SLINE_EINVAL) && G > 1;
        if (apart) {
            // device memory ran short for the batch as a whole, or one of its
            // graphs was refused: run its queries one at a time (a single
            // graph needs no combined output), so that each query gets the
            // status of its own plain build
            for (int32_t g = 0; g < G; ++g) {
                outs[g] = sline_edges{};
                qst[g] = sline_build_batch(W.ctx, 1, &Hs[g], &ss[g], &ds[g], flags, &outs[g]);
            }
            st = SLINE_OK;
            for (int32_t g = 0; g < G; ++g)
                if (qst[g] != SLINE_OK) st = qst[g];
        }
        const int64_t t_done = now_ns();
        if (S->log) {
            int64_t pairs = 0, big = 0;
            for (int32_t g = 0; g < G; ++g) {
                pairs += qst[g] == SLINE_OK ? outs[g].n_pairs : 0;
                big += Hs[g].n_edges >= 500000;
            }
            sline_stats ps{};
            (void)sline_last_stats(W.ctx, &ps);
            int64_t c1[5];
            size_t cache_bytes = 0;
            {
                std::lock_guard<std::mutex> lk(S->cache.mu);
                cache_bytes = S->cache.total;
                c1[0] = S->cache.n_malloc;
                c1[1] = S->cache.n_malloc_fail;
                c1[2] = S->cache.n_free;
                c1[3] = S->cache.ns_malloc;
                c1[4] = S->cache.ns_free;
            }
            // cache figures are process-wide: they include other workers' calls meanwhile
            fprintf(stderr, "sline-server: worker %d batch of %d%s (%lld large, est %.2f GB) status %d "
                    "pairs %lld %.1f ms [transpose %.1f prepare %.1f count %.1f fill %.1f; "
                    "hipMalloc %lld (%lld failed) %.1f ms, hipFree %lld %.1f ms, cache %.1f GB]\n",
                    wi, G, apart ? " run apart" : "", (long long)big, est / 1e9, st, (long long)pairs, (t_done - t_run) / 1e6,
                    ps.ms_transpose, ps.ms_prepare, ps.ms_count, ps.ms_fill,
                    (long long)(c1[0] - c0[0]), (long long)(c1[1] - c0[1]), (c1[3] - c0[3]) / 1e6,
                    (long long)(c1[2] - c0[2]), (c1[4] - c0[4]) / 1e6, cache_bytes / 1e9);
        }
        std::string err = st == SLINE_OK ? std::string() : std::string(sline_last_error(W.ctx));
        {
            std::lock_guard<std::mutex> lk(S->mu);
            // keep the results that can answer later queries of their graph
            // and side; the builds of this batch are no longer running
            for (int32_t g = 0; g < G; ++g) {
                if (qst[g] == SLINE_OK) keep_result(S, gs[g], ds[g], ss[g], outs[g]);
                auto bt = S->building.find({gs[g], ds[g]});
                if (bt != S->building.end() && bt->second == ss[g]) S->building.erase(bt);
            }
        }
        // queries built at a smaller s than they asked for: their answer is
        // the build filtered to their s (the build itself stays only as a
        // kept result, if it was kept)
        std::vector<sline_edges> fouts(G);
        for (int32_t g = 0; g < G; ++g) {
            if (qst[g] != SLINE_OK || want[g] == ss[g]) continue;
            fouts[g] = sline_edges{};
            const sline_status fs = sline_filter(W.ctx, &outs[g], want[g], 0, &fouts[g]);
            if (fs != SLINE_OK) err = sline_last_error(W.ctx);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                free_arrays(S, outs[g]);
            }
            outs[g] = fouts[g];
            qst[g] = fs;
            if (fs != SLINE_OK && st == SLINE_OK) st = fs;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (int32_t g = 0; g < G; ++g) {
                Query &q = S->queries[batch[g]];
                q.info.status = qst[g];
                q.info.t_done_ns = now_ns();
                if (qst[g] == SLINE_OK) {
                    q.out = outs[g];
                    q.info.n_pairs = outs[g].n_pairs;
                    S->held += result_bytes(outs[g]);
                }
                q.done = true;
            }
            for (int32_t r = 0; r < R; ++r) {
                Query &q = S->queries[reuse[r]];
                q.info.status = rst[r];
                q.info.t_done_ns = t_done;
                if (rst[r] == SLINE_OK) {
                    q.out = routs[r];
                    q.info.n_pairs = routs[r].n_pairs;
                    S->held += result_bytes(routs[r]);
                }
                q.done = true;
            }
            if (st != SLINE_OK) S->last_error = err;
            else if (!rerr.empty()) S->last_error = rerr;
            S->in_flight -= est;
            S->running -= 1;
        }
        S->cv.notify_all();
    }
}

// Results live in the server's cache; a release returns them to it unless a
// kept entry still shares them (caller holds S->mu).
void free_arrays(sline_server *S, const sline_edges &e) {
    unref(S, e.a);
    unref(S, e.b);
    unref(S, e.w);
}

}  // namespace

extern "C" {

sline_status sline_server_create(sline_server **srv, int device, int64_t hbm_budget_bytes,
                                 int32_t max_batch, int32_t n_workers) {
    if (!srv || hbm_budget_bytes <= 0 || max_batch < 1 || n_workers < 1 || n_workers > 16)
        return SLINE_EINVAL;
    *srv = nullptr;
    sline_server *S = new (std::nothrow) sline_server();
    if (!S) return SLINE_ENOMEM;
    S->device = device;
    S->budget = hbm_budget_bytes;
    S->max_batch = max_batch;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        return SLINE_EDEVICE;
    }
    sline_allocator al{};
    al.alloc = cache_alloc;
    al.free = cache_free;
    al.user = &S->cache;
    S->log = getenv("SLINE_SERVER_LOG") != nullptr;
    S->reuse_cap = std::min<int64_t>(hbm_budget_bytes / 4, (int64_t)32 << 30);
    S->reuse_min_nnz = (int64_t)1 << 20;
    // the budget and the kept results, mapped once (fresh device memory costs
    // far more than a build)
    S->cache.reserve((size_t)(hbm_budget_bytes + S->reuse_cap));
    S->workers.resize(n_workers);
    for (auto &W : S->workers) {
        if (hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            sline_server_destroy(S);
            return SLINE_EDEVICE;
        }
        const sline_status st = sline_create(&W.ctx, device, W.stream, &al);
        if (st != SLINE_OK) {
            sline_server_destroy(S);
            return st;
        }
    }
    try {
        for (int i = 0; i < n_workers; ++i) S->workers[i].th = std::thread(worker_loop, S, i);
    } catch (...) {
        sline_server_destroy(S);
        return SLINE_ENOMEM;
    }
    *srv = S;
    return SLINE_OK;
}

sline_status sline_server_register(sline_server *S, sline_csr H, int32_t *graph_id) {
    if (!S || !graph_id || H.n_edges < 0 || H.n_vertices < 0 || (H.n_edges > 0 && !H.row_ptr))
        return SLINE_EINVAL;
    Graph g;
    g.H = H;
    // W_1 of both sides from the item sizes and the vertex degrees
    std::vector<int32_t> rp((size_t)H.n_edges + 1, 0);
    if (H.n_edges > 0 &&
        hipMemcpy(rp.data(), H.row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return SLINE_EDEVICE;
    }
    g.nnz = rp.back();
    // the full CSR rules of sline_build, so that a malformed graph is refused
    // here rather than failing every batch its queries would join
    if (rp[0] != 0 || g.nnz < 0 || (g.nnz > 0 && (!H.col_idx || H.n_vertices == 0)))
        return SLINE_EINVAL;
    for (int32_t e = 0; e < H.n_edges; ++e) {
        const double k = rp[e + 1] - rp[e];
        if (k < 0) return SLINE_EINVAL;
        g.w1[1] += k * (k - 1) / 2;
    }
    if (g.nnz > 0) {
        std::vector<int32_t> col((size_t)g.nnz);
        if (hipMemcpy(col.data(), H.col_idx, sizeof(int32_t) * col.size(), hipMemcpyDeviceToHost) !=
            hipSuccess) {
            (void)hipGetLastError();
            return SLINE_EDEVICE;
        }
        std::vector<int32_t> deg((size_t)H.n_vertices, 0);
        for (int32_t e = 0; e < H.n_edges; ++e) {
            for (int32_t k = rp[e]; k < rp[e + 1]; ++k) {
                const int32_t v = col[k];
                if (v < 0 || v >= H.n_vertices) return SLINE_EINVAL;
                if (k > rp[e] && v <= col[k - 1]) return SLINE_EINVAL;  // rows are sets, ascending
                deg[v] += 1;
            }
        }
        for (int32_t d : deg) g.w1[0] += (double)d * (d - 1) / 2;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    *graph_id = (int32_t)S->graphs.size();
    S->graphs.push_back(g);
    return SLINE_OK;
}

sline_status sline_server_submit(sline_server *S, int32_t graph_id, int32_t s, int32_t dual,
                                 int64_t *ticket) {
    if (!S || !ticket || s < 1 || (dual != 0 && dual != 1)) return SLINE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (graph_id < 0 || graph_id >= (int32_t)S->graphs.size()) return SLINE_EINVAL;
        Query q;
        q.ticket = S->next_ticket++;
        q.graph = graph_id;
        q.s = s;
        q.dual = dual;
        q.est = estimate(S->graphs[graph_id], s, dual);
        q.s_build = s;
        q.info.t_submit_ns = now_ns();
        q.info.status = SLINE_EBUSY;
        *ticket = q.ticket;
        S->queries.emplace(q.ticket, q);
        S->queue.push_back(q.ticket);
    }
    S->cv.notify_all();
    return SLINE_OK;
}

sline_status sline_server_poll(sline_server *S, int64_t ticket, sline_edges *out,
                               sline_query_info *info) {
    if (!S || !out) return SLINE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->queries.find(ticket);
    if (it == S->queries.end()) return SLINE_EINVAL;
    if (!it->second.done) return SLINE_EBUSY;
    const Query q = it->second;
    S->queries.erase(it);
    if (info) *info = q.info;
    if (q.info.status != SLINE_OK) return q.info.status;
    *out = q.out;
    out->capacity = 0;
    // the arrays stay owned by the server until sline_server_release
    return SLINE_OK;
}

sline_status sline_server_release(sline_server *S, sline_edges *out) {
    if (!S || !out) return SLINE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (out->a || out->b) S->held = std::max<int64_t>(0, S->held - result_bytes(*out));
        free_arrays(S, *out);
    }
    S->cv.notify_all();  // admission may have waited on the released memory
    out->a = out->b = out->w = nullptr;
    out->n_pairs = 0;
    return SLINE_OK;
}

sline_status sline_server_set_reuse(sline_server *S, int64_t cache_bytes, int64_t min_nnz,
                                    uint32_t flags) {
    if (!S || cache_bytes < 0 || min_nnz < 0 || (flags & ~(uint32_t)SLINE_REUSE_LOOKAHEAD))
        return SLINE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->reuse_cap = cache_bytes;
        S->reuse_min_nnz = min_nnz;
        S->lookahead = (flags & SLINE_REUSE_LOOKAHEAD) != 0;
        evict_kept(S, cache_bytes);
    }
    // map room for the budget and the kept results up front (if the device
    // has it to spare)
    size_t have = 0;
    {
        std::lock_guard<std::mutex> lk(S->cache.mu);
        have = S->cache.total;
    }
    const size_t want = (size_t)(S->budget + cache_bytes);
    if (have < want) S->cache.reserve(want - have);
    return SLINE_OK;
}

sline_status sline_server_reuse_stats(sline_server *S, int64_t *reused, int64_t *kept,
                                      int64_t *kept_bytes) {
    if (!S) return SLINE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (reused) *reused = S->n_reused;
    if (kept) *kept = S->n_kept;
    if (kept_bytes) *kept_bytes = S->kept_bytes;
    return SLINE_OK;
}

sline_status sline_server_pending(sline_server *S, int64_t *queued, int32_t *running) {
    if (!S) return SLINE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (queued) *queued = (int64_t)S->queue.size();
    if (running) *running = S->running;
    return SLINE_OK;
}

const char *sline_server_last_error(sline_server *S) {
    return S ? S->last_error.c_str() : "no server";
}

void sline_server_destroy(sline_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto &W : S->workers)
        if (W.th.joinable()) W.th.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto &kv : S->queries)
            if (kv.second.done) free_arrays(S, kv.second.out);
        for (auto &kv : S->kept) free_arrays(S, kv.second.e);
        S->kept.clear();
    }
    for (auto &W : S->workers) {
        if (W.ctx) sline_destroy(W.ctx);
        if (W.stream) (void)hipStreamDestroy(W.stream);
    }
    (void)hipDeviceSynchronize();
    S->cache.destroy();
    delete S;
}

}  // extern "C"
