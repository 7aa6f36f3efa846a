/*
 * CPU oracle for the s-line graph L_s(H) of a hypergraph.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this file; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg use it.  It shares no
 * code, header or table with the device path.
 *
 * What it computes (paper, Sec. III): items are the hyperedges e_1..e_m of H
 * (or, for the dual hypergraph H*, its vertices); two distinct items a, b are
 * joined in L_s(H) when their overlap w_ab = |S_a intersect S_b| is at least
 * s, s >= 1.  Output: every (a, b, w_ab) with a < b and w_ab >= s, sorted by
 * (a, b).  Integer arithmetic only; there is nothing to round.
 *
 * Two oracles, both written from the paper, both plain and slow:
 *
 *  O1  oracle_naive_rows -- the definition itself, as the naive algorithm of
 *      Sec. IV-A states it: for every pair of items, count the common members
 *      by a two-pointer merge of the two sorted member lists and keep the pair
 *      when the count reaches s.  Only the upper triangle b > a is visited
 *      (Sec. IV-C, applied to every variant in Sec. V-C), so exactly N(N-1)/2
 *      intersections are made when the size skip is off (Table I counts
 *      m(m-1)/2 of them for the naive method).
 *
 *  O3  oracle_wedge_rows -- the alternative algorithm of Sec. IV-B with the
 *      visited array of Sec. IV-C turned into a counter: for item a, every
 *      vertex v of S_a and every item b containing v with b > a adds one to
 *      cnt[b]; afterwards cnt[b] = w_ab for every b sharing a member with a.
 *      Items smaller than s are skipped on both ends (degree-based pruning,
 *      Sec. IV-C), which cannot change the result since w_ab <= min(|S_a|,
 *      |S_b|).  It is exact (not an approximation) and is checked against O1.
 *
 *  O2  oracle_alg_h_rows -- the efficient algorithm with heuristics of
 *      Sec. IV-C (the second printed algorithm) with each heuristic as a
 *      switch, so that the variants f0..f4 of Sec. V-C (Table III) run as
 *      printed: degree-based pruning of e_i and e_j (size < s), skipping
 *      hyperedges already visited for e_i, and a set intersection that stops
 *      once s common members are found (short-circuit).  The strictly upper
 *      triangle is kept in every variant, as Sec. V-C states.  L_s is a set,
 *      so a pair met again through another shared vertex (visited skipping
 *      off) is added once.  Output weights are exact: when the intersection
 *      stopped early, an accepted pair's overlap is counted in full.  The
 *      stats count the set intersections made (Table I's measure of work).
 *
 *  oracle_components -- the connected components of the graph L_s (the
 *      s-connected components of Table I): union-find over the edge list,
 *      every component labelled by its smallest item id.
 *
 * Parallelism: items are dealt cyclically to threads (Sec. IV-F, cyclic
 * range); each thread keeps its own row buffers and the rows are concatenated
 * in item order at the end, so the result does not depend on the thread count.
 *
 * Ownership: results are malloc'd here and released with oracle_free_pairs.
 * Errors: functions return 0 on success, -1 on bad arguments, -2 when memory
 * runs out.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;   /* number of pairs */
    int32_t *a;  /* first item (a < b)   */
    int32_t *b;  /* second item          */
    int32_t *w;  /* overlap |S_a & S_b|  */
} oracle_pairs;

typedef struct {
    int64_t n_pairs;        /* |L_s| over the rows visited              */
    int64_t sum_w;          /* sum of w over those pairs                 */
    uint64_t digest;        /* sum over pairs of mix(a, b, w), mod 2^64  */
    int64_t wedges;         /* O3: increments made;  O1, O2: 0           */
    int64_t intersections;  /* O1, O2: set intersections made; O3: 0     */
} oracle_stats;

/* ------------------------------------------------------------ utilities */

/* Order-independent digest term of one output triple (test bookkeeping). */
uint64_t oracle_mix(int32_t a, int32_t b, int32_t w) {
    uint64_t x = (uint64_t)(uint32_t)a * 0x9E3779B97F4A7C15ull;
    x ^= (uint64_t)(uint32_t)b * 0xC2B2AE3D27D4EB4Full;
    x ^= (uint64_t)(uint32_t)w * 0x165667B19E3779F9ull;
    x ^= x >> 31;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    return x;
}

/* Transpose by counting sort: item lists of the dual (Sec. III).  rpT has
 * n+1 entries, colT has nnz; rows of the result come out sorted because the
 * input is scanned in row order. */
int oracle_transpose(const int32_t *rp, const int32_t *col, int32_t m, int32_t n,
                     int32_t *rpT, int32_t *colT) {
    if (m < 0 || n < 0 || !rp || !rpT) return -1;
    int64_t nnz = rp[m];
    memset(rpT, 0, sizeof(int32_t) * ((size_t)n + 1));
    for (int64_t k = 0; k < nnz; ++k) {
        int32_t v = col[k];
        if (v < 0 || v >= n) return -1;
        rpT[v + 1] += 1;
    }
    for (int32_t v = 0; v < n; ++v) rpT[v + 1] += rpT[v];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!fill) return -2;
    memcpy(fill, rpT, sizeof(int32_t) * ((size_t)n + 1));
    for (int32_t i = 0; i < m; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) colT[fill[col[k]]++] = i;
    free(fill);
    return 0;
}

/* Number of common members of two sorted lists (two-pointer merge). */
static int32_t merge_count(const int32_t *x, int32_t nx, const int32_t *y, int32_t ny) {
    int32_t i = 0, j = 0, c = 0;
    while (i < nx && j < ny) {
        if (x[i] < y[j]) ++i;
        else if (y[j] < x[i]) ++j;
        else { ++c; ++i; ++j; }
    }
    return c;
}

/* --------------------------------------------------- per-thread buffers */

typedef struct {
    int64_t n, cap;
    int32_t *b, *w;
} rowbuf;

static int rb_push(rowbuf *r, int32_t b, int32_t w) {
    if (r->n == r->cap) {
        int64_t nc = r->cap ? 2 * r->cap : 1024;
        int32_t *nb = (int32_t *)realloc(r->b, sizeof(int32_t) * nc);
        if (!nb) return -2;
        r->b = nb;
        int32_t *nw = (int32_t *)realloc(r->w, sizeof(int32_t) * nc);
        if (!nw) return -2;
        r->w = nw;
        r->cap = nc;
    }
    r->b[r->n] = b;
    r->w[r->n] = w;
    r->n++;
    return 0;
}

typedef struct {
    const int32_t *rp, *col;   /* item lists */
    const int32_t *rpT, *colT; /* membership lists (O2, O3) */
    int32_t N, s, skip_small, keep;
    int32_t variant;           /* O2: heuristics on (ORACLE_H_* bits) */
    const int32_t *rows;       /* rows to visit, NULL = all */
    int64_t nrows;
    int tid, nthreads;
    rowbuf out;                /* this thread's pairs, rows in visit order */
    int64_t *row_count;        /* per visited row index: pairs emitted */
    oracle_stats st;
    int err;
} job;

static void record(job *J, int64_t ri, int32_t a, int32_t b, int32_t w) {
    J->st.n_pairs++;
    J->st.sum_w += w;
    J->st.digest += oracle_mix(a, b, w);
    J->row_count[ri]++;
    if (J->keep && rb_push(&J->out, b, w)) J->err = -2;
}

static void *naive_worker(void *p) {
    job *J = (job *)p;
    for (int64_t ri = J->tid; ri < J->nrows && !J->err; ri += J->nthreads) {
        int32_t a = J->rows ? J->rows[ri] : (int32_t)ri;
        const int32_t *Sa = J->col + J->rp[a];
        int32_t na = J->rp[a + 1] - J->rp[a];
        for (int32_t b = a + 1; b < J->N; ++b) {
            const int32_t *Sb = J->col + J->rp[b];
            int32_t nb = J->rp[b + 1] - J->rp[b];
            if (J->skip_small && (na < J->s || nb < J->s)) continue;
            J->st.intersections++;
            int32_t w = merge_count(Sa, na, Sb, nb);
            if (w >= J->s) record(J, ri, a, b, w);
        }
    }
    return NULL;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t u = *(const int32_t *)x, v = *(const int32_t *)y;
    return (u > v) - (u < v);
}

static void *wedge_worker(void *p) {
    job *J = (job *)p;
    int32_t *cnt = (int32_t *)calloc((size_t)J->N + 1, sizeof(int32_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * ((size_t)J->N + 1));
    if (!cnt || !touched) { J->err = -2; free(cnt); free(touched); return NULL; }
    for (int64_t ri = J->tid; ri < J->nrows && !J->err; ri += J->nthreads) {
        int32_t a = J->rows ? J->rows[ri] : (int32_t)ri;
        int32_t na = J->rp[a + 1] - J->rp[a];
        if (na < J->s) continue;                       /* prune e_a */
        int64_t nt = 0;
        for (int32_t k = J->rp[a]; k < J->rp[a + 1]; ++k) {
            int32_t v = J->col[k];
            for (int32_t t = J->rpT[v]; t < J->rpT[v + 1]; ++t) {
                int32_t b = J->colT[t];
                if (b <= a) continue;                  /* upper triangle only */
                if (J->rp[b + 1] - J->rp[b] < J->s) continue; /* prune e_b */
                if (cnt[b] == 0) touched[nt++] = b;
                cnt[b] += 1;
                J->st.wedges++;
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < nt; ++t) {
            int32_t b = touched[t];
            if (cnt[b] >= J->s) record(J, ri, a, b, cnt[b]);
            cnt[b] = 0;
        }
    }
    free(cnt);
    free(touched);
    return NULL;
}

/* O2 heuristic switches (Sec. IV-C). */
enum { ORACLE_H_PRUNE = 1, ORACLE_H_VISITED = 2, ORACLE_H_SHORT = 4 };

/* At least s common members?  The merge stops as soon as s are found. */
static int merge_at_least(const int32_t *x, int32_t nx, const int32_t *y, int32_t ny, int32_t s) {
    int32_t i = 0, j = 0, c = 0;
    while (i < nx && j < ny) {
        if (x[i] < y[j]) ++i;
        else if (y[j] < x[i]) ++j;
        else {
            if (++c >= s) return 1;
            ++i;
            ++j;
        }
    }
    return 0;
}

static void *alg_h_worker(void *p) {
    job *J = (job *)p;
    const int prune = J->variant & ORACLE_H_PRUNE;
    const int visit = J->variant & ORACLE_H_VISITED;
    const int shortc = J->variant & ORACLE_H_SHORT;
    uint8_t *visited = (uint8_t *)calloc((size_t)J->N + 1, 1);
    int64_t cap = 1024;
    int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);  /* accepted j of e_i */
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * ((size_t)J->N + 1));
    if (!visited || !acc || !touched) {
        J->err = -2;
        free(visited); free(acc); free(touched);
        return NULL;
    }
    for (int64_t ri = J->tid; ri < J->nrows && !J->err; ri += J->nthreads) {
        const int32_t i = J->rows ? J->rows[ri] : (int32_t)ri;
        const int32_t *Si = J->col + J->rp[i];
        const int32_t ni = J->rp[i + 1] - J->rp[i];
        if (prune && ni < J->s) continue;              /* degree-based pruning of e_i */
        int64_t nt = 0, na = 0;
        for (int32_t k = J->rp[i]; k < J->rp[i + 1]; ++k) {
            const int32_t v = J->col[k];
            for (int32_t t = J->rpT[v]; t < J->rpT[v + 1]; ++t) {
                const int32_t j = J->colT[t];
                if (i >= j) continue;                  /* strictly upper triangle */
                const int32_t *Sj = J->col + J->rp[j];
                const int32_t nj = J->rp[j + 1] - J->rp[j];
                if (prune && nj < J->s) continue;      /* degree-based pruning of e_j */
                if (visit) {                           /* skip hyperedges already visited */
                    if (visited[j]) continue;
                    visited[j] = 1;
                    touched[nt++] = j;
                }
                J->st.intersections++;
                const int ok = shortc ? merge_at_least(Si, ni, Sj, nj, J->s)
                                      : merge_count(Si, ni, Sj, nj) >= J->s;
                if (ok) {
                    if (na == cap) {
                        int32_t *g = (int32_t *)realloc(acc, sizeof(int32_t) * (size_t)(2 * cap));
                        if (!g) { J->err = -2; break; }
                        acc = g;
                        cap *= 2;
                    }
                    acc[na++] = j;
                }
            }
            if (J->err) break;
        }
        for (int64_t t = 0; t < nt; ++t) visited[touched[t]] = 0;
        /* L_s is a set: each accepted e_j once, in id order, with its overlap */
        qsort(acc, (size_t)na, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < na && !J->err; ++t) {
            if (t > 0 && acc[t] == acc[t - 1]) continue;
            const int32_t j = acc[t];
            record(J, ri, i, j, merge_count(Si, ni, J->col + J->rp[j], J->rp[j + 1] - J->rp[j]));
        }
    }
    free(visited);
    free(acc);
    free(touched);
    return NULL;
}

/* Run `worker` over the rows with `nthreads` cyclic workers and gather. */
static int run(void *(*worker)(void *), const int32_t *rp, const int32_t *col,
               const int32_t *rpT, const int32_t *colT, int32_t N, int32_t s,
               int32_t skip_small, int32_t variant, const int32_t *rows, int64_t nrows,
               int nthreads, int keep, oracle_pairs *out, oracle_stats *stats) {
    if (N < 0 || s < 1 || (N > 0 && !rp) || nthreads < 1) return -1;
    if (!rows) nrows = N;
    for (int64_t r = 0; rows && r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= N) return -1;
    job *J = (job *)calloc((size_t)nthreads, sizeof(job));
    int64_t *row_count = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!J || !row_count || !th) { free(J); free(row_count); free(th); return -2; }
    for (int t = 0; t < nthreads; ++t) {
        J[t].rp = rp; J[t].col = col; J[t].rpT = rpT; J[t].colT = colT;
        J[t].N = N; J[t].s = s; J[t].skip_small = skip_small; J[t].keep = keep;
        J[t].variant = variant;
        J[t].rows = rows; J[t].nrows = nrows; J[t].tid = t; J[t].nthreads = nthreads;
        J[t].row_count = row_count;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &J[t]);
    worker(&J[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);

    int err = 0;
    oracle_stats tot = {0, 0, 0, 0, 0};
    for (int t = 0; t < nthreads; ++t) {
        if (J[t].err) err = J[t].err;
        tot.n_pairs += J[t].st.n_pairs;
        tot.sum_w += J[t].st.sum_w;
        tot.digest += J[t].st.digest;
        tot.wedges += J[t].st.wedges;
        tot.intersections += J[t].st.intersections;
    }
    if (!err && keep) {
        out->n = tot.n_pairs;
        size_t bytes = sizeof(int32_t) * (size_t)(tot.n_pairs ? tot.n_pairs : 1);
        out->a = (int32_t *)malloc(bytes);
        out->b = (int32_t *)malloc(bytes);
        out->w = (int32_t *)malloc(bytes);
        if (!out->a || !out->b || !out->w) err = -2;
        int64_t *cursor = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
        if (!cursor) err = -2;
        int64_t o = 0;
        for (int64_t ri = 0; !err && ri < nrows; ++ri) {
            job *Jt = &J[ri % nthreads];
            int32_t a = rows ? rows[ri] : (int32_t)ri;
            int64_t c = row_count[ri], base = cursor[ri % nthreads];
            for (int64_t q = 0; q < c; ++q) {
                out->a[o] = a;
                out->b[o] = Jt->out.b[base + q];
                out->w[o] = Jt->out.w[base + q];
                ++o;
            }
            cursor[ri % nthreads] += c;
        }
        free(cursor);
        if (err) { free(out->a); free(out->b); free(out->w); out->a = out->b = out->w = NULL; }
    }
    if (stats) *stats = tot;
    for (int t = 0; t < nthreads; ++t) { free(J[t].out.b); free(J[t].out.w); }
    free(J); free(row_count); free(th);
    return err;
}

/* O1.  Items are the rows of (rp, col), N of them.  rows/nrows select which
 * items a are visited (rows may be NULL for all, and must be ascending for the
 * output to be in canonical order); every b > a is compared.  skip_small turns
 * on the exactness-preserving size skip.  keep = 0 returns only stats. */
int oracle_naive_rows(const int32_t *rp, const int32_t *col, int32_t N, int32_t s,
                      int32_t skip_small, const int32_t *rows, int64_t nrows,
                      int nthreads, int keep, oracle_pairs *out, oracle_stats *stats) {
    return run(naive_worker, rp, col, NULL, NULL, N, s, skip_small, 0, rows, nrows,
               nthreads, keep, out, stats);
}

/* O3.  Items are the rows of (rp, col), N of them; (rpT, colT) lists, for each
 * member, the items containing it (the transpose, rows ascending). */
int oracle_wedge_rows(const int32_t *rp, const int32_t *col, const int32_t *rpT,
                      const int32_t *colT, int32_t N, int32_t s, const int32_t *rows,
                      int64_t nrows, int nthreads, int keep, oracle_pairs *out,
                      oracle_stats *stats) {
    if (!rpT && N > 0) return -1;
    return run(wedge_worker, rp, col, rpT, colT, N, s, 1, 0, rows, nrows, nthreads, keep,
               out, stats);
}

/* O2.  As O3's arguments, plus `variant`: the ORACLE_H_* heuristics that are
 * on (7 = f0, PRUNE = f1, VISITED = f2, SHORT = f3, 0 = f4 of Table III). */
int oracle_alg_h_rows(const int32_t *rp, const int32_t *col, const int32_t *rpT,
                      const int32_t *colT, int32_t N, int32_t s, int32_t variant,
                      const int32_t *rows, int64_t nrows, int nthreads, int keep,
                      oracle_pairs *out, oracle_stats *stats) {
    if ((!rpT && N > 0) || variant < 0 || variant > 7) return -1;
    return run(alg_h_worker, rp, col, rpT, colT, N, s, 0, variant, rows, nrows, nthreads, keep,
               out, stats);
}

/* Connected components of the graph on items 0..N-1 with edges (a[e], b[e]):
 * comp[x] = the smallest item of x's component (an item without edges is
 * its own component).  Union-find with path halving; a union links the
 * larger root under the smaller, so a component's root is its minimum. */
static int32_t uf_find(int32_t *parent, int32_t x) {
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

int oracle_components(int32_t N, const int32_t *a, const int32_t *b, int64_t n, int32_t *comp) {
    if (N < 0 || n < 0 || (N > 0 && !comp) || (n > 0 && (!a || !b))) return -1;
    for (int32_t x = 0; x < N; ++x) comp[x] = x;
    for (int64_t e = 0; e < n; ++e) {
        if (a[e] < 0 || a[e] >= N || b[e] < 0 || b[e] >= N) return -1;
        int32_t ra = uf_find(comp, a[e]), rb = uf_find(comp, b[e]);
        if (ra == rb) continue;
        if (ra < rb) comp[rb] = ra;
        else comp[ra] = rb;
    }
    for (int32_t x = 0; x < N; ++x) comp[x] = uf_find(comp, x);
    return 0;
}

void oracle_free_pairs(oracle_pairs *p) {
    if (!p) return;
    free(p->a); free(p->b); free(p->w);
    p->a = p->b = p->w = NULL;
    p->n = 0;
}
