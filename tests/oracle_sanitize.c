/*
 * Driver that runs the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by test_oracle_sanitized.py with gcc).
 *
 * It draws small random hypergraphs (empty rows, a one-vertex universe,
 * full rows), runs the transpose, O1 and O3 at several s, thread counts and
 * row selections, with and without kept pairs, and checks that O1 and O3
 * agree and that bad arguments are refused.  Any sanitizer report ends the
 * run with a non-zero status; a mismatch returns 1.
 */
#include "../oracle/sline_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x243F6A8885A308D3ull;

static uint32_t next_u32(void) { /* 64-bit LCG (Knuth's MMIX constants), high half */
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(rng_state >> 32);
}

static int32_t below(int32_t n) { return n > 0 ? (int32_t)(next_u32() % (uint32_t)n) : 0; }

/* m rows over n vertices; row sizes from 0 to n, members sorted and distinct */
static void random_graph(int32_t m, int32_t n, int32_t **rp_out, int32_t **col_out) {
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t cap = 16, nnz = 0;
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    rp[0] = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t k = below(4) == 0 ? below(n + 1) : below(n < 5 ? n + 1 : 5);
        for (int32_t v = 0; v < n; ++v) perm[v] = v;
        for (int32_t j = 0; j < k; ++j) { /* partial Fisher-Yates */
            int32_t r = j + below(n - j);
            int32_t t = perm[j]; perm[j] = perm[r]; perm[r] = t;
        }
        qsort(perm, (size_t)k, sizeof(int32_t), cmp_i32);
        if (nnz + k > cap) {
            while (nnz + k > cap) cap *= 2;
            col = (int32_t *)realloc(col, sizeof(int32_t) * (size_t)cap);
        }
        memcpy(col + nnz, perm, sizeof(int32_t) * (size_t)k);
        nnz += k;
        rp[i + 1] = (int32_t)nnz;
    }
    free(perm);
    *rp_out = rp;
    *col_out = col;
}

static int same_pairs(const oracle_pairs *x, const oracle_pairs *y) {
    if (x->n != y->n) return 0;
    for (int64_t k = 0; k < x->n; ++k)
        if (x->a[k] != y->a[k] || x->b[k] != y->b[k] || x->w[k] != y->w[k]) return 0;
    return 1;
}

int main(void) {
    const int32_t shapes[][2] = {{0, 3}, {1, 1}, {2, 1}, {5, 4}, {40, 7}, {120, 30}, {200, 60}};
    int checks = 0;
    for (size_t t = 0; t < sizeof(shapes) / sizeof(shapes[0]); ++t) {
        const int32_t m = shapes[t][0], n = shapes[t][1];
        int32_t *rp, *col;
        random_graph(m, n, &rp, &col);
        int32_t *rpT = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
        int32_t *colT = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[m] > 0 ? rp[m] : 1));
        if (oracle_transpose(rp, col, m, n, rpT, colT) != 0) return 1;
        int32_t rows[3] = {0, m / 2, m - 1};
        int64_t nrows = m >= 3 ? 3 : 0;
        for (int32_t s = 1; s <= 4; ++s) {
            for (int threads = 1; threads <= 4; threads += 3) {
                for (int sel = 0; sel < 2; ++sel) {
                    const int32_t *r = sel ? rows : NULL;
                    const int64_t nr = sel ? nrows : 0;
                    if (sel && nrows == 0) continue;
                    oracle_pairs p1 = {0, NULL, NULL, NULL}, p3 = {0, NULL, NULL, NULL};
                    oracle_stats s1, s3, s0;
                    if (oracle_naive_rows(rp, col, m, s, 0, r, nr, threads, 1, &p1, &s1)) return 1;
                    if (oracle_wedge_rows(rp, col, rpT, colT, m, s, r, nr, threads, 1, &p3, &s3))
                        return 1;
                    if (oracle_naive_rows(rp, col, m, s, 1, r, nr, threads, 0, NULL, &s0)) return 1;
                    if (!same_pairs(&p1, &p3) || s1.digest != s3.digest || s0.digest != s1.digest) {
                        printf("mismatch m=%d n=%d s=%d threads=%d sel=%d\n", m, n, s, threads, sel);
                        return 1;
                    }
                    oracle_free_pairs(&p1);
                    oracle_free_pairs(&p3);
                    ++checks;
                }
            }
        }
        /* bad arguments are refused */
        oracle_stats st;
        int32_t bad_row = m;
        if (oracle_naive_rows(rp, col, -1, 1, 0, NULL, 0, 1, 0, NULL, &st) != -1) return 1;
        if (oracle_naive_rows(rp, col, m, 0, 0, NULL, 0, 1, 0, NULL, &st) != -1) return 1;
        if (oracle_naive_rows(rp, col, m, 1, 0, &bad_row, 1, 1, 0, NULL, &st) != -1) return 1;
        if (oracle_naive_rows(rp, col, m, 1, 0, NULL, 0, 0, 0, NULL, &st) != -1) return 1;
        if (m > 0 && oracle_wedge_rows(rp, col, NULL, NULL, m, 1, NULL, 0, 1, 0, NULL, &st) != -1)
            return 1;
        if (n > 0 && rp[m] > 0) { /* a member id out of range */
            int32_t keep = col[0];
            col[0] = n;
            if (oracle_transpose(rp, col, m, n, rpT, colT) != -1) return 1;
            col[0] = keep;
        }
        free(rp); free(col); free(rpT); free(colT);
    }
    printf("ok %d checks\n", checks);
    return 0;
}
