/* Exercises every entry point of the CPU oracle on small seeded graphs, so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer sees
 * each code path once: load and export, a batch (with no-op deletions and
 * insertions, and a batch rejected for an id out of range), Static,
 * Naive-dynamic, Dynamic Frontier, Dynamic Traversal and the marking
 * helpers.  Built and run by test_oracle_sanitized.py; prints "ok" and
 * exits 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dfpr_oracle.h"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

/* xorshift64* (Vigna, 2016) */
static uint32_t next_u32(void)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static double sum_of(const double *x, int32_t n)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; i++) s += x[i];
    return s;
}

static double linf(const double *a, const double *b, int32_t n)
{
    double d = 0.0;
    for (int32_t i = 0; i < n; i++) d = fmax(d, fabs(a[i] - b[i]));
    return d;
}

static int run(int32_t n, int64_t m)
{
    const double alpha = 0.85, tol = 1e-10, ftol = 1e-15;
    int32_t *src = malloc((size_t)m * 4), *dst = malloc((size_t)m * 4);
    for (int64_t i = 0; i < m; i++) {
        src[i] = (int32_t)(next_u32() % (uint32_t)n);
        dst[i] = (int32_t)(next_u32() % (uint32_t)n);
    }
    oracle_graph *g = NULL;
    CHECK(oracle_load_graph(n, m, src, dst, &g) == 0 && g);
    int32_t nn = 0;
    int64_t mm = 0;
    CHECK(oracle_graph_info(g, &nn, &mm) == 0 && nn == n && mm >= n && mm <= m + n);

    /* batch: deletions of listed edges (self-loops and repeats among them
     * are no-ops), insertions of random pairs (present ones are no-ops) */
    const int64_t nd = 20, ni = 40;
    int32_t ds[20], dd[20], is[40], id[40];
    for (int64_t i = 0; i < nd; i++) {
        if (m == 0) {
            ds[i] = dd[i] = 0;          /* the self-loop, never deleted */
            continue;
        }
        const int64_t k = (int64_t)(next_u32() % (uint32_t)m);
        ds[i] = src[k];
        dd[i] = dst[k];
    }
    for (int64_t i = 0; i < ni; i++) {
        is[i] = (int32_t)(next_u32() % (uint32_t)n);
        id[i] = (int32_t)(next_u32() % (uint32_t)n);
    }

    int64_t *off = malloc((size_t)(n + 1) * 8);
    int32_t *idx = malloc((size_t)(mm + ni) * 4);
    double *R0 = malloc((size_t)n * 8), *R1 = malloc((size_t)n * 8);
    double *Rs = malloc((size_t)n * 8), *Rn = malloc((size_t)n * 8);
    double *Rt = malloc((size_t)n * 8), *dr = malloc((size_t)n * 8);
    uint8_t *f0 = malloc((size_t)n), *f1 = malloc((size_t)n), *f2 = malloc((size_t)n);
    oracle_stats st;

    for (int o = 0; o < 2; o++) {
        CHECK(oracle_export_csr(g, o, off, idx) == 0);
        CHECK(off[0] == 0 && off[n] == mm);
    }
    CHECK(oracle_pagerank_static(g, alpha, tol, 500, R0, &st) == 0 && st.converged);
    CHECK(fabs(sum_of(R0, n) - 1.0) < 1e-8);

    /* a batch with an id out of range is rejected and changes nothing */
    int32_t bad = n;
    int64_t applied[2] = {-1, -1};
    CHECK(oracle_apply_batch(g, 0, NULL, NULL, 1, is, &bad, applied) != 0);
    CHECK(oracle_graph_info(g, &nn, &mm) == 0 && off[n] == mm);

    CHECK(oracle_apply_batch(g, nd, ds, dd, ni, is, id, applied) == 0);
    CHECK(applied[0] >= 0 && applied[0] <= nd && applied[1] >= 0 && applied[1] <= ni);
    CHECK(oracle_graph_info(g, &nn, &mm) == 0);
    CHECK(oracle_export_csr(g, 1, off, idx) == 0 && off[n] == mm);

    CHECK(oracle_mark_initial_csr(n, off, idx, nd, ds, dd, ni, is, id, f0) == 0);
    CHECK(oracle_pagerank_dynamic_frontier(g, alpha, tol, ftol, 500, nd, ds, dd, ni, is, id,
                                           R0, R1, &st, f1, f2, dr) == 0 && st.converged);
    for (int32_t v = 0; v < n; v++) CHECK(dr[v] >= 0.0 && (f2[v] || dr[v] == 0.0));
    for (int32_t v = 0; v < n; v++) CHECK(f1[v] == f0[v] && (!f1[v] || f2[v]));
    CHECK(oracle_pagerank_static(g, alpha, tol, 500, Rs, &st) == 0 && st.converged);
    CHECK(linf(R1, Rs, n) < 1e-8);
    CHECK(oracle_pagerank_naive_dynamic(g, alpha, tol, 500, R0, Rn, &st) == 0 && st.converged);
    CHECK(linf(Rn, Rs, n) < 1e-8);

    for (int32_t v = 0; v < n; v++) dr[v] = fabs(R1[v] - R0[v]);
    CHECK(oracle_expand_csr(n, off, idx, f0, dr, ftol, f2) == 0);
    for (int32_t v = 0; v < n; v++) CHECK(!f0[v] || f2[v]);

    CHECK(oracle_mark_reachable_csr(n, off, idx, nd, ds, dd, ni, is, id, f1) == 0);
    CHECK(oracle_pagerank_dynamic_traversal(g, alpha, tol, 500, nd, ds, dd, ni, is, id, R0,
                                            Rt, &st, f2) == 0 && st.converged);
    for (int32_t v = 0; v < n; v++) CHECK(f1[v] == f2[v]);
    CHECK(linf(Rt, Rs, n) < 1e-8);

    /* an empty batch: the previous ranks come back after one iteration */
    CHECK(oracle_pagerank_dynamic_frontier(g, alpha, tol, ftol, 500, 0, NULL, NULL, 0, NULL,
                                           NULL, Rs, R1, &st, NULL, NULL, NULL) == 0);
    CHECK(st.iterations == 1 && st.converged && linf(R1, Rs, n) == 0.0);

    oracle_free_graph(g);
    free(src);
    free(dst);
    free(off);
    free(idx);
    free(R0);
    free(R1);
    free(Rs);
    free(Rn);
    free(Rt);
    free(dr);
    free(f0);
    free(f1);
    free(f2);
    return 0;
}

int main(void)
{
    CHECK(oracle_num_threads() >= 1);
    CHECK(run(300, 2400) == 0);
    CHECK(run(1, 0) == 0);          /* one vertex: only its self-loop */
    CHECK(run(2000, 30000) == 0);
    printf("ok\n");
    return 0;
}
