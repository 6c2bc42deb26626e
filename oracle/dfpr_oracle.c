/*
 * CPU reference ("oracle") for Dynamic Frontier PageRank — TEST
 * INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).
 * Shares no code with the GPU library.  See dfpr_oracle.h for the
 * interface; every function below names the passage of the paper it
 * follows.
 *
 * Representation: the edge set E is a sorted array of 64-bit keys
 * (u << 32 | v).  The out-CSR and in-CSR are rebuilt from it after every
 * change, so both are always exactly the set E with rows sorted by id.
 */
#include "dfpr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct oracle_graph {
    int32_t n;
    int64_t m;          /* |E|, self-loops included                     */
    uint64_t *keys;     /* sorted, distinct (u << 32 | v)               */
    int64_t *out_off;   /* n + 1                                        */
    int32_t *out_idx;   /* m: out(u) = out_idx[out_off[u] .. out_off[u+1]) */
    int64_t *in_off;    /* n + 1                                        */
    int32_t *in_idx;    /* m: in(v)  = in_idx[in_off[v] .. in_off[v+1])    */
};

#define KEY(u, v) (((uint64_t)(uint32_t)(u) << 32) | (uint64_t)(uint32_t)(v))
#define KEY_SRC(k) ((int32_t)((k) >> 32))
#define KEY_DST(k) ((int32_t)((k) & 0xffffffffu))

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Sort keys and drop repeats; returns the new length. */
static int64_t sort_unique(uint64_t *k, int64_t len)
{
    if (len == 0) return 0;
    qsort(k, (size_t)len, sizeof(uint64_t), cmp_u64);
    int64_t w = 1;
    for (int64_t i = 1; i < len; i++)
        if (k[i] != k[w - 1]) k[w++] = k[i];
    return w;
}

/* Rebuild both CSRs from the sorted key array.  The out-CSR rows come out
 * sorted because the keys are sorted by (u, v).  The in-CSR is a stable
 * counting sort of the keys by v; visiting keys in increasing u keeps each
 * in-row sorted. */
static int rebuild_csr(oracle_graph *g)
{
    int32_t n = g->n;
    int64_t m = g->m;
    free(g->out_off); free(g->out_idx); free(g->in_off); free(g->in_idx);
    g->out_off = calloc((size_t)n + 1, sizeof(int64_t));
    g->in_off = calloc((size_t)n + 1, sizeof(int64_t));
    g->out_idx = malloc((size_t)(m ? m : 1) * sizeof(int32_t));
    g->in_idx = malloc((size_t)(m ? m : 1) * sizeof(int32_t));
    int64_t *cursor = malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!g->out_off || !g->in_off || !g->out_idx || !g->in_idx || !cursor) {
        free(cursor);
        return -3;
    }
    for (int64_t e = 0; e < m; e++) {
        g->out_off[KEY_SRC(g->keys[e]) + 1]++;
        g->in_off[KEY_DST(g->keys[e]) + 1]++;
    }
    for (int32_t v = 0; v < n; v++) {
        g->out_off[v + 1] += g->out_off[v];
        g->in_off[v + 1] += g->in_off[v];
    }
    for (int64_t e = 0; e < m; e++) g->out_idx[e] = KEY_DST(g->keys[e]);
    memcpy(cursor, g->in_off, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {
        int32_t u = KEY_SRC(g->keys[e]), v = KEY_DST(g->keys[e]);
        g->in_idx[cursor[v]++] = u;
    }
    free(cursor);
    return 0;
}

static int ids_ok(int32_t n, int64_t len, const int32_t *a, const int32_t *b)
{
    for (int64_t i = 0; i < len; i++)
        if (a[i] < 0 || a[i] >= n || b[i] < 0 || b[i] >= n) return 0;
    return 1;
}

/* Section 3.1: the graph gets a self-loop on every vertex (dead-end
 * removal); E is a set, so repeated input edges count once. */
int oracle_load_graph(int32_t n, int64_t m, const int32_t *src,
                      const int32_t *dst, oracle_graph **out)
{
    if (!out || n <= 0 || m < 0 || (m > 0 && (!src || !dst))) return -1;
    if (!ids_ok(n, m, src, dst)) return -2;
    oracle_graph *g = calloc(1, sizeof(*g));
    if (!g) return -3;
    g->n = n;
    g->keys = malloc((size_t)(m + n) * sizeof(uint64_t));
    if (!g->keys) { free(g); return -3; }
    for (int64_t i = 0; i < m; i++) g->keys[i] = KEY(src[i], dst[i]);
    for (int32_t v = 0; v < n; v++) g->keys[m + v] = KEY(v, v);
    g->m = sort_unique(g->keys, m + n);
    int rc = rebuild_csr(g);
    if (rc) { oracle_free_graph(g); return rc; }
    *out = g;
    return 0;
}

void oracle_free_graph(oracle_graph *g)
{
    if (!g) return;
    free(g->keys); free(g->out_off); free(g->out_idx);
    free(g->in_off); free(g->in_idx);
    free(g);
}

int oracle_graph_info(const oracle_graph *g, int32_t *n, int64_t *m)
{
    if (!g) return -1;
    if (n) *n = g->n;
    if (m) *m = g->m;
    return 0;
}

int oracle_export_csr(const oracle_graph *g, int orientation,
                      int64_t *offsets, int32_t *idx)
{
    if (!g || !offsets || !idx) return -1;
    const int64_t *off = orientation ? g->out_off : g->in_off;
    const int32_t *ix = orientation ? g->out_idx : g->in_idx;
    memcpy(offsets, off, ((size_t)g->n + 1) * sizeof(int64_t));
    memcpy(idx, ix, (size_t)g->m * sizeof(int32_t));
    return 0;
}

/* Section 3.2: Delta- = E^{t-1} \ E^t and Delta+ = E^t \ E^{t-1}, so
 * E^t = (E^{t-1} \ Delta-) U Delta+.  Section 5.1.4: self-loops stay on
 * every vertex, so deleting one does nothing. */
int oracle_apply_batch(oracle_graph *g,
                       int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                       int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                       int64_t applied[2])
{
    if (!g || n_del < 0 || n_ins < 0) return -1;
    if ((n_del && (!del_src || !del_dst)) || (n_ins && (!ins_src || !ins_dst))) return -1;
    if (!ids_ok(g->n, n_del, del_src, del_dst) || !ids_ok(g->n, n_ins, ins_src, ins_dst))
        return -2;
    uint64_t *dk = malloc((size_t)(n_del ? n_del : 1) * sizeof(uint64_t));
    uint64_t *ik = malloc((size_t)(n_ins ? n_ins : 1) * sizeof(uint64_t));
    uint64_t *nk = malloc((size_t)(g->m + n_ins + 1) * sizeof(uint64_t));
    if (!dk || !ik || !nk) { free(dk); free(ik); free(nk); return -3; }
    int64_t nd = 0;
    for (int64_t i = 0; i < n_del; i++)
        if (del_src[i] != del_dst[i]) dk[nd++] = KEY(del_src[i], del_dst[i]);
    nd = sort_unique(dk, nd);
    for (int64_t i = 0; i < n_ins; i++) ik[i] = KEY(ins_src[i], ins_dst[i]);
    int64_t ni = sort_unique(ik, n_ins);

    /* E' = E \ D (merge of two sorted lists) */
    int64_t a = 0, b = 0, w = 0, eff_del = 0;
    while (a < g->m) {
        while (b < nd && dk[b] < g->keys[a]) b++;
        if (b < nd && dk[b] == g->keys[a]) { eff_del++; a++; continue; }
        g->keys[w++] = g->keys[a++];
    }
    int64_t m1 = w;
    /* E'' = E' U I (merge) */
    a = 0; b = 0; w = 0;
    int64_t eff_ins = 0;
    while (a < m1 || b < ni) {
        if (b >= ni || (a < m1 && g->keys[a] < ik[b])) nk[w++] = g->keys[a++];
        else if (a >= m1 || ik[b] < g->keys[a]) { nk[w++] = ik[b++]; eff_ins++; }
        else { nk[w++] = g->keys[a++]; b++; }
    }
    free(g->keys);
    g->keys = nk;
    g->m = w;
    free(dk); free(ik);
    if (applied) { applied[0] = eff_del; applied[1] = eff_ins; }
    return rebuild_csr(g);
}

/* Eq. 1 at vertex v, as printed: alpha times the sum over the
 * in-neighbours u of R[u] / |out(u)|, plus (1 - alpha)/|V|.  The sum runs
 * over the in-row in ascending id order. */
static double eq1(const oracle_graph *g, const double *R, int32_t v, double alpha)
{
    double sum = 0.0;
    for (int64_t k = g->in_off[v]; k < g->in_off[v + 1]; k++) {
        const int32_t u = g->in_idx[k];
        sum += R[u] / (double)(g->out_off[u + 1] - g->out_off[u]);
    }
    return alpha * sum + (1.0 - alpha) / (double)g->n;
}

/* Work done by one sweep. */
typedef struct {
    double linf;       /* largest |new - old| over the vertices swept */
    int64_t verts;     /* vertices swept                              */
    int64_t edges;     /* their in-edges                              */
} sweep_result;

/* One synchronous sweep (Section 4.2): new ranks of the vertices picked by
 * `pick` (every vertex when it is NULL) are computed from `cur` with Eq. 1
 * and written to `out`; `cur` is not written.  `change` (nullable)
 * receives |new - old| of each picked vertex and 0 elsewhere. */
static sweep_result sweep(const oracle_graph *g, const uint8_t *pick, const double *cur,
                          double *out, double *change, double alpha)
{
    sweep_result res = {0.0, 0, 0};
    double linf = 0.0;
    int64_t verts = 0, edges = 0;
#pragma omp parallel for schedule(dynamic, 2048) reduction(max : linf) reduction(+ : verts, edges)
    for (int32_t v = 0; v < g->n; v++) {
        if (pick && !pick[v]) {
            if (change) change[v] = 0.0;
            continue;
        }
        const double r = eq1(g, cur, v, alpha);
        const double d = fabs(r - cur[v]);
        out[v] = r;
        if (change) change[v] = d;
        linf = d > linf ? d : linf;
        verts += 1;
        edges += g->in_off[v + 1] - g->in_off[v];
    }
    res.linf = linf;
    res.verts = verts;
    res.edges = edges;
    return res;
}

/* Power iteration over all vertices from the start vector R (n entries,
 * overwritten with the result): sweeps alternate between two vectors until
 * the L-inf change is at most tol (Section 3.1). */
static int power_iterate(const oracle_graph *g, double alpha, double tol,
                         int32_t max_iters, double *R, oracle_stats *st)
{
    int32_t n = g->n;
    double *other = malloc((size_t)n * sizeof(double));
    if (!other) return -3;
    double *cur = R, *nxt = other;
    oracle_stats s = {0};
    while (s.iterations < max_iters) {
        const sweep_result w = sweep(g, NULL, cur, nxt, NULL, alpha);
        double *t = cur; cur = nxt; nxt = t;
        s.iterations += 1;
        s.final_linf = w.linf;
        s.vertices_processed += w.verts;
        s.edges_processed += w.edges;
        if (w.linf <= tol) { s.converged = 1; break; }
    }
    if (cur != R) memcpy(R, cur, (size_t)n * sizeof(double));
    free(other);
    s.affected_initial = s.affected_final = n;
    if (st) *st = s;
    return 0;
}

/* Section 3.1: every vertex starts at 1/n. */
int oracle_pagerank_static(const oracle_graph *g, double alpha, double tol,
                           int32_t max_iters, double *ranks_out,
                           oracle_stats *st)
{
    if (!g || !ranks_out || max_iters < 0) return -1;
    for (int32_t v = 0; v < g->n; v++) ranks_out[v] = 1.0 / (double)g->n;
    return power_iterate(g, alpha, tol, max_iters, ranks_out, st);
}

/* Section 3.3.1: start from the previous snapshot's ranks and process all
 * vertices. */
int oracle_pagerank_naive_dynamic(const oracle_graph *g, double alpha,
                                  double tol, int32_t max_iters,
                                  const double *prev, double *ranks_out,
                                  oracle_stats *st)
{
    if (!g || !prev || !ranks_out || max_iters < 0) return -1;
    if (ranks_out != prev) memcpy(ranks_out, prev, (size_t)g->n * sizeof(double));
    return power_iterate(g, alpha, tol, max_iters, ranks_out, st);
}

/* Section 4.1.1, first rule (Algorithm 1, initial marking): for each
 * deleted or inserted edge (u, v), the out-neighbours of u in G^{t-1} and
 * in G^t are affected.  G^{t-1}.out(u) differs from G^t.out(u) only by the
 * batch edges leaving u (Section 3.2), so the union is G^t.out(u) plus the
 * v of each deletion.  The set of batch sources is collected first, then
 * each source's out-row is marked once, then the deletion targets. */
int oracle_mark_initial_csr(int32_t n, const int64_t *out_off,
                            const int32_t *out_idx,
                            int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                            int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                            uint8_t *flags)
{
    if (n <= 0 || !out_off || !flags || n_del < 0 || n_ins < 0) return -1;
    if ((n_del && (!del_src || !del_dst)) || (n_ins && (!ins_src || !ins_dst))) return -1;
    if (!ids_ok(n, n_del, del_src, del_dst) || !ids_ok(n, n_ins, ins_src, ins_dst))
        return -2;
    uint8_t *is_source = calloc((size_t)n, 1);
    if (!is_source) return -3;
    for (int64_t i = 0; i < n_del; i++) is_source[del_src[i]] = 1;
    for (int64_t i = 0; i < n_ins; i++) is_source[ins_src[i]] = 1;
    memset(flags, 0, (size_t)n);
    for (int32_t u = 0; u < n; u++) {
        if (!is_source[u]) continue;
        for (int64_t k = out_off[u]; k < out_off[u + 1]; k++) flags[out_idx[k]] = 1;
    }
    for (int64_t i = 0; i < n_del; i++) flags[del_dst[i]] = 1;
    free(is_source);
    return 0;
}

/* Section 4.1.1, second rule (Algorithm 1, incremental marking): an
 * affected vertex whose rank moved by more than the frontier tolerance
 * marks its out-neighbours.  Marks go to a separate vector and take effect
 * from the next iteration. */
int oracle_expand_csr(int32_t n, const int64_t *out_off, const int32_t *out_idx,
                      const uint8_t *affected, const double *dr,
                      double frontier_tol, uint8_t *next)
{
    if (n <= 0 || !out_off || !affected || !dr || !next) return -1;
    memcpy(next, affected, (size_t)n);
#pragma omp parallel for schedule(dynamic, 2048)
    for (int32_t v = 0; v < n; v++) {
        if (!(affected[v] && dr[v] > frontier_tol)) continue;
        for (int64_t k = out_off[v]; k < out_off[v + 1]; k++) {
            int32_t w = out_idx[k];
#pragma omp atomic write
            next[w] = 1;
        }
    }
    return 0;
}

/* Dynamic Frontier (Section 4.1, Algorithm 1) in the synchronous form of
 * Section 4.2.  The ranks start at the previous snapshot's and the marks at
 * the initial marking.  Each iteration sweeps the marked vertices with
 * Eq. 1 from the current vector into the other one; a swept vertex whose
 * rank moved by more than frontier_tol marks its out-neighbours in G^t for
 * the next iteration (marks only grow within one update); the loop ends
 * once the largest move of the sweep is at most tol, or after max_iters
 * sweeps.  Between sweeps the two vectors agree on every vertex not swept,
 * so a sweep need only write the vertices it processes. */
int oracle_pagerank_dynamic_frontier(
    const oracle_graph *g, double alpha, double tol, double frontier_tol,
    int32_t max_iters,
    int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
    int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
    const double *prev, double *ranks_out, oracle_stats *st,
    uint8_t *affected_initial, uint8_t *affected_final, double *largest_change)
{
    if (!g || !prev || !ranks_out || max_iters < 0) return -1;
    int32_t n = g->n;
    uint8_t *marks = malloc((size_t)n);
    uint8_t *grown = malloc((size_t)n);
    double *A = malloc((size_t)n * sizeof(double));
    double *B = malloc((size_t)n * sizeof(double));
    double *change = malloc((size_t)n * sizeof(double));
    if (!marks || !grown || !A || !B || !change) {
        free(marks); free(grown); free(A); free(B); free(change);
        return -3;
    }
    int rc = oracle_mark_initial_csr(n, g->out_off, g->out_idx, n_del, del_src,
                                     del_dst, n_ins, ins_src, ins_dst, marks);
    if (rc) { free(marks); free(grown); free(A); free(B); free(change); return rc; }
    memcpy(A, prev, (size_t)n * sizeof(double));
    memcpy(B, prev, (size_t)n * sizeof(double));
    oracle_stats s = {0};
    for (int32_t v = 0; v < n; v++) s.affected_initial += marks[v];
    if (affected_initial) memcpy(affected_initial, marks, (size_t)n);
    if (largest_change) memset(largest_change, 0, (size_t)n * sizeof(double));

    double *cur = A, *nxt = B;
    while (s.iterations < max_iters) {
        const sweep_result w = sweep(g, marks, cur, nxt, change, alpha);
        oracle_expand_csr(n, g->out_off, g->out_idx, marks, change, frontier_tol, grown);
        if (largest_change)
            for (int32_t v = 0; v < n; v++)
                if (change[v] > largest_change[v]) largest_change[v] = change[v];
        /* the vector just read becomes the next output: copy in the swept
         * vertices so that the two agree again everywhere */
#pragma omp parallel for schedule(static)
        for (int32_t v = 0; v < n; v++)
            if (marks[v]) cur[v] = nxt[v];
        double *t = cur; cur = nxt; nxt = t;
        uint8_t *tm = marks; marks = grown; grown = tm;
        s.iterations += 1;
        s.final_linf = w.linf;
        s.vertices_processed += w.verts;
        s.edges_processed += w.edges;
        if (w.linf <= tol) { s.converged = 1; break; }
    }
    memcpy(ranks_out, cur, (size_t)n * sizeof(double));
    for (int32_t v = 0; v < n; v++) s.affected_final += marks[v];
    if (affected_final) memcpy(affected_final, marks, (size_t)n);
    if (st) *st = s;
    free(marks); free(grown); free(A); free(B); free(change);
    return 0;
}

/* Section 3.3.2 (Dynamic Traversal): for each deleted or inserted edge
 * (u, v), every vertex reachable from u in G^{t-1} or in G^t is affected.
 * Reachability is taken in the union graph G^{t-1} union G^t, whose
 * out-edges are those of G^t plus the deleted batch edges (every deleted
 * edge leaves a batch source); a vertex reaches itself.  A plain
 * first-in-first-out breadth-first search. */
static int cmp_pair(const void *a, const void *b)
{
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int oracle_mark_reachable_csr(int32_t n, const int64_t *out_off,
                              const int32_t *out_idx,
                              int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                              int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                              uint8_t *flags)
{
    if (n <= 0 || !out_off || !flags || n_del < 0 || n_ins < 0) return -1;
    if ((n_del && (!del_src || !del_dst)) || (n_ins && (!ins_src || !ins_dst))) return -1;
    if (!ids_ok(n, n_del, del_src, del_dst) || !ids_ok(n, n_ins, ins_src, ins_dst))
        return -2;
    /* deleted edges as (source, target) keys, sorted, for their out-rows */
    int64_t *del = malloc((size_t)(n_del ? n_del : 1) * sizeof(int64_t));
    int32_t *queue = malloc((size_t)n * sizeof(int32_t));
    if (!del || !queue) { free(del); free(queue); return -3; }
    for (int64_t i = 0; i < n_del; i++) del[i] = (int64_t)del_src[i] * n + del_dst[i];
    qsort(del, (size_t)n_del, sizeof(int64_t), cmp_pair);
    memset(flags, 0, (size_t)n);
    int64_t head = 0, tail = 0;
    for (int64_t i = 0; i < n_del + n_ins; i++) {
        int32_t u = i < n_del ? del_src[i] : ins_src[i - n_del];
        if (!flags[u]) { flags[u] = 1; queue[tail++] = u; }
    }
    while (head < tail) {
        int32_t x = queue[head++];
        for (int64_t k = out_off[x]; k < out_off[x + 1]; k++) {
            int32_t w = out_idx[k];
            if (!flags[w]) { flags[w] = 1; queue[tail++] = w; }
        }
        /* deleted edges leaving x: first key >= x * n */
        int64_t lo = 0, hi = n_del;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (del[mid] < (int64_t)x * n) lo = mid + 1; else hi = mid;
        }
        for (int64_t j = lo; j < n_del && del[j] / n == x; j++) {
            int32_t w = (int32_t)(del[j] % n);
            if (!flags[w]) { flags[w] = 1; queue[tail++] = w; }
        }
    }
    free(del);
    free(queue);
    return 0;
}

/* Dynamic Traversal PageRank (Section 3.3.2) in the synchronous form: mark
 * the reachable set once, then iterate Eq. 1 over the marked vertices only,
 * from the previous ranks, until Delta R <= tol.  No vertex is marked
 * during the iterations. */
int oracle_pagerank_dynamic_traversal(
    const oracle_graph *g, double alpha, double tol, int32_t max_iters,
    int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
    int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
    const double *prev, double *ranks_out, oracle_stats *st, uint8_t *affected)
{
    if (!g || !prev || !ranks_out || max_iters < 0) return -1;
    int32_t n = g->n;
    uint8_t *aff = malloc((size_t)n);
    double *R = malloc((size_t)n * sizeof(double));
    double *Rn = malloc((size_t)n * sizeof(double));
    if (!aff || !R || !Rn) { free(aff); free(R); free(Rn); return -3; }
    int rc = oracle_mark_reachable_csr(n, g->out_off, g->out_idx, n_del, del_src, del_dst,
                                       n_ins, ins_src, ins_dst, aff);
    if (rc) { free(aff); free(R); free(Rn); return rc; }
    memcpy(R, prev, (size_t)n * sizeof(double));
    memcpy(Rn, prev, (size_t)n * sizeof(double));
    oracle_stats s = {0};
    for (int32_t v = 0; v < n; v++) s.affected_initial += aff[v];
    s.affected_final = s.affected_initial;
    if (affected) memcpy(affected, aff, (size_t)n);
    /* the marked set never changes, so the swept vertices are the same
     * every time and the two vectors agree on the others throughout */
    double *cur = R, *nxt = Rn;
    while (s.iterations < max_iters) {
        const sweep_result w = sweep(g, aff, cur, nxt, NULL, alpha);
        double *t = cur; cur = nxt; nxt = t;
        s.iterations += 1;
        s.final_linf = w.linf;
        s.vertices_processed += w.verts;
        s.edges_processed += w.edges;
        if (w.linf <= tol) { s.converged = 1; break; }
    }
    memcpy(ranks_out, cur, (size_t)n * sizeof(double));
    if (st) *st = s;
    free(aff); free(R); free(Rn);
    return 0;
}
