/* A plain C99 caller of the library's C-ABI (include/dfpr.h), with no Python
 * and no torch in the process: it loads a graph, computes Static PageRank,
 * applies one batch and updates the ranks with Dynamic Frontier and
 * Naive-dynamic (Sections 3.1, 3.3.1 and 4.1), and exercises the error
 * returns of the boundary.
 *
 *   abi_c_driver EDGES BATCH OUT_PREFIX
 *
 * EDGES: "n m" then m lines "u v".  BATCH: "n_del n_ins" then n_del
 * deletions and n_ins insertions, one "u v" per line.  Writes
 * OUT_PREFIX.static, OUT_PREFIX.df and OUT_PREFIX.naive (n ranks each, one
 * per line, %.17g) and prints one line of counts.  Exits non-zero with a
 * message on the first unexpected status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dfpr.h"

static int fail(const char *what, int rc)
{
    const char *msg = dfpr_last_error();
    fprintf(stderr, "abi_c_driver: %s returned %d (%s)\n", what, rc, msg ? msg : "");
    return 1;
}

static int read_pairs(FILE *f, int64_t k, int32_t *a, int32_t *b)
{
    for (int64_t i = 0; i < k; i++)
        if (fscanf(f, "%d %d", &a[i], &b[i]) != 2) return -1;
    return 0;
}

static int write_ranks(const char *prefix, const char *tag, const double *r, int32_t n)
{
    char path[4096];
    snprintf(path, sizeof path, "%s.%s", prefix, tag);
    FILE *f = fopen(path, "w");
    if (!f) return -1;
    for (int32_t i = 0; i < n; i++) fprintf(f, "%.17g\n", r[i]);
    return fclose(f);
}

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: abi_c_driver EDGES BATCH OUT_PREFIX\n");
        return 2;
    }
    int32_t n = 0;
    int64_t m = 0, nd = 0, ni = 0;
    FILE *fe = fopen(argv[1], "r");
    if (!fe || fscanf(fe, "%d %ld", &n, &m) != 2 || n <= 0 || m < 0) {
        fprintf(stderr, "abi_c_driver: cannot read %s\n", argv[1]);
        return 2;
    }
    int32_t *src = malloc((size_t)(m ? m : 1) * sizeof *src);
    int32_t *dst = malloc((size_t)(m ? m : 1) * sizeof *dst);
    if (!src || !dst || read_pairs(fe, m, src, dst)) return 2;
    fclose(fe);
    FILE *fb = fopen(argv[2], "r");
    if (!fb || fscanf(fb, "%ld %ld", &nd, &ni) != 2 || nd < 0 || ni < 0) {
        fprintf(stderr, "abi_c_driver: cannot read %s\n", argv[2]);
        return 2;
    }
    int32_t *ds = malloc((size_t)(nd ? nd : 1) * sizeof *ds);
    int32_t *dd = malloc((size_t)(nd ? nd : 1) * sizeof *dd);
    int32_t *is = malloc((size_t)(ni ? ni : 1) * sizeof *is);
    int32_t *id = malloc((size_t)(ni ? ni : 1) * sizeof *id);
    if (!ds || !dd || !is || !id || read_pairs(fb, nd, ds, dd) || read_pairs(fb, ni, is, id))
        return 2;
    fclose(fb);

    /* error returns: no graph, and a graph with an id outside [0, n) */
    dfpr_params p;
    dfpr_params_default(&p);
    double dummy = 0.0;
    int rc = dfpr_pagerank_static(NULL, &p, &dummy, NULL);
    if (rc != DFPR_E_ARG) return fail("static on a NULL graph", rc);
    dfpr_graph *g = NULL;
    int32_t bad_src = n, bad_dst = 0;
    rc = dfpr_load_graph(n, 1, &bad_src, &bad_dst, &g);
    if (rc != DFPR_E_RANGE || g) return fail("load with an id out of range", rc);
    if (!dfpr_last_error() || !dfpr_last_error()[0]) return fail("last_error after a failure", rc);

    rc = dfpr_load_graph(n, m, src, dst, &g);
    if (rc) return fail("load_graph", rc);
    int32_t gn = 0;
    int64_t m0 = 0;
    rc = dfpr_graph_info(g, &gn, &m0);
    if (rc || gn != n) return fail("graph_info", rc);

    double *r0 = malloc((size_t)n * sizeof *r0);
    double *rdf = malloc((size_t)n * sizeof *rdf);
    double *rnv = malloc((size_t)n * sizeof *rnv);
    if (!r0 || !rdf || !rnv) return 2;
    dfpr_stats st0, stdf, stnv;
    rc = dfpr_pagerank_static(g, &p, r0, &st0);
    if (rc || !st0.converged) return fail("pagerank_static", rc);

    /* a batch with an id out of range is refused and changes nothing */
    int64_t applied[2] = {-1, -1};
    rc = dfpr_apply_batch(g, 0, NULL, NULL, 1, &bad_src, &bad_dst, applied);
    int64_t m1 = 0;
    if (rc != DFPR_E_RANGE || dfpr_graph_info(g, &gn, &m1) || m1 != m0)
        return fail("apply_batch with an id out of range", rc);

    rc = dfpr_apply_batch(g, nd, ds, dd, ni, is, id, applied);
    if (rc) return fail("apply_batch", rc);
    rc = dfpr_pagerank_dynamic_frontier(g, &p, nd, ds, dd, ni, is, id, r0, rdf, &stdf);
    if (rc || !stdf.converged) return fail("pagerank_dynamic_frontier", rc);
    rc = dfpr_pagerank_naive_dynamic(g, &p, r0, rnv, &stnv);
    if (rc || !stnv.converged) return fail("pagerank_naive_dynamic", rc);
    int64_t m2 = 0;
    rc = dfpr_graph_info(g, &gn, &m2);
    if (rc) return fail("graph_info", rc);
    dfpr_free_graph(g);

    if (write_ranks(argv[3], "static", r0, n) || write_ranks(argv[3], "df", rdf, n) ||
        write_ranks(argv[3], "naive", rnv, n)) {
        fprintf(stderr, "abi_c_driver: cannot write under %s\n", argv[3]);
        return 2;
    }
    printf("n %d m %ld applied %ld %ld m_after %ld static_it %d df_it %d df_affected %ld naive_it %d\n",
           n, m0, applied[0], applied[1], m2, st0.iterations, stdf.iterations,
           stdf.affected_final, stnv.iterations);
    free(src); free(dst); free(ds); free(dd); free(is); free(id);
    free(r0); free(rdf); free(rnv);
    return 0;
}
