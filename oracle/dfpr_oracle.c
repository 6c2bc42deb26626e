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

/* Eq. 1 for one vertex, in the order of Algorithm 1's rank loop:
 * r = (1 - alpha)/|V|, then r += alpha * R[u] / |out(u)| for u in in(v). */
static double rank_of(const oracle_graph *g, const double *R, int32_t v,
                      double alpha)
{
    double r = (1.0 - alpha) / (double)g->n;
    for (int64_t k = g->in_off[v]; k < g->in_off[v + 1]; k++) {
        int32_t u = g->in_idx[k];
        double outdeg = (double)(g->out_off[u + 1] - g->out_off[u]);
        r += alpha * R[u] / outdeg;
    }
    return r;
}

/* Power iteration over all vertices from the start vector R (n entries,
 * overwritten with the result); synchronous: reads R, writes a second
 * vector, then swaps (Section 4.2). */
static int power_iterate(const oracle_graph *g, double alpha, double tol,
                         int32_t max_iters, double *R, oracle_stats *st)
{
    int32_t n = g->n;
    double *Rn = malloc((size_t)n * sizeof(double));
    if (!Rn) return -3;
    double *cur = R, *nxt = Rn;
    oracle_stats s = {0};
    for (int32_t it = 0; it < max_iters; it++) {
        double dR = 0.0;
        int64_t edges = 0;
#pragma omp parallel for schedule(dynamic, 2048) reduction(max : dR) reduction(+ : edges)
        for (int32_t v = 0; v < n; v++) {
            double r = rank_of(g, cur, v, alpha);
            double d = fabs(r - cur[v]);
            nxt[v] = r;
            if (d > dR) dR = d;
            edges += g->in_off[v + 1] - g->in_off[v];
        }
        double *t = cur; cur = nxt; nxt = t;
        s.iterations = it + 1;
        s.final_linf = dR;
        s.vertices_processed += n;
        s.edges_processed += edges;
        if (dR <= tol) { s.converged = 1; break; }
    }
    if (cur != R) memcpy(R, cur, (size_t)n * sizeof(double));
    free(Rn);
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
 * v of each deletion. */
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
    memset(flags, 0, (size_t)n);
    for (int64_t i = 0; i < n_del + n_ins; i++) {
        int32_t u = i < n_del ? del_src[i] : ins_src[i - n_del];
        for (int64_t k = out_off[u]; k < out_off[u + 1]; k++) flags[out_idx[k]] = 1;
        if (i < n_del) flags[del_dst[i]] = 1;
    }
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

/* Algorithm 1 in the synchronous form of Section 4.2:
 *   R <- R^{t-1}; mark initial affected;
 *   repeat up to max_iters times:
 *     Delta R <- 0
 *     for each affected v: r from Eq. 1 over G^t.in(v);
 *        dr = |r - R[v]|; R'[v] = r; Delta R = max(Delta R, dr);
 *        if dr > frontier_tol: mark G^t.out(v)
 *     stop if Delta R <= tol.
 * R' starts equal to R and only affected rows are written, so after the
 * swap the unaffected rows hold their unchanged ranks.  Marks made during
 * an iteration are processed from the next iteration on; marks are never
 * cleared within one update. */
int oracle_pagerank_dynamic_frontier(
    const oracle_graph *g, double alpha, double tol, double frontier_tol,
    int32_t max_iters,
    int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
    int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
    const double *prev, double *ranks_out, oracle_stats *st,
    uint8_t *affected_initial, uint8_t *affected_final)
{
    if (!g || !prev || !ranks_out || max_iters < 0) return -1;
    int32_t n = g->n;
    uint8_t *aff = malloc((size_t)n);
    uint8_t *nxt = malloc((size_t)n);
    double *R = malloc((size_t)n * sizeof(double));
    double *Rn = malloc((size_t)n * sizeof(double));
    double *dr = malloc((size_t)n * sizeof(double));
    if (!aff || !nxt || !R || !Rn || !dr) {
        free(aff); free(nxt); free(R); free(Rn); free(dr);
        return -3;
    }
    int rc = oracle_mark_initial_csr(n, g->out_off, g->out_idx, n_del, del_src,
                                     del_dst, n_ins, ins_src, ins_dst, aff);
    if (rc) { free(aff); free(nxt); free(R); free(Rn); free(dr); return rc; }
    memcpy(R, prev, (size_t)n * sizeof(double));
    memcpy(Rn, prev, (size_t)n * sizeof(double));
    oracle_stats s = {0};
    for (int32_t v = 0; v < n; v++) s.affected_initial += aff[v];
    if (affected_initial) memcpy(affected_initial, aff, (size_t)n);

    double *cur = R, *out = Rn;
    for (int32_t it = 0; it < max_iters; it++) {
        double dR = 0.0;
        int64_t edges = 0, verts = 0;
#pragma omp parallel for schedule(dynamic, 2048) reduction(max : dR) reduction(+ : edges, verts)
        for (int32_t v = 0; v < n; v++) {
            dr[v] = 0.0;
            if (!aff[v]) continue;
            double r = rank_of(g, cur, v, alpha);
            double d = fabs(r - cur[v]);
            out[v] = r;
            dr[v] = d;
            if (d > dR) dR = d;
            verts += 1;
            edges += g->in_off[v + 1] - g->in_off[v];
        }
        /* incremental marking into a separate vector */
        oracle_expand_csr(n, g->out_off, g->out_idx, aff, dr, frontier_tol, nxt);
        double *t = cur; cur = out; out = t;
        /* the buffer just read becomes the next output: bring its affected
         * rows up to date so that every unaffected row matches */
#pragma omp parallel for schedule(static)
        for (int32_t v = 0; v < n; v++)
            if (aff[v]) out[v] = cur[v];
        uint8_t *tf = aff; aff = nxt; nxt = tf;
        s.iterations = it + 1;
        s.final_linf = dR;
        s.vertices_processed += verts;
        s.edges_processed += edges;
        if (dR <= tol) { s.converged = 1; break; }
    }
    memcpy(ranks_out, cur, (size_t)n * sizeof(double));
    for (int32_t v = 0; v < n; v++) s.affected_final += aff[v];
    if (affected_final) memcpy(affected_final, aff, (size_t)n);
    if (st) *st = s;
    free(aff); free(nxt); free(R); free(Rn); free(dr);
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
    double *cur = R, *out = Rn;
    for (int32_t it = 0; it < max_iters; it++) {
        double dR = 0.0;
        int64_t edges = 0, verts = 0;
#pragma omp parallel for schedule(dynamic, 2048) reduction(max : dR) reduction(+ : edges, verts)
        for (int32_t v = 0; v < n; v++) {
            if (!aff[v]) continue;
            double r = rank_of(g, cur, v, alpha);
            double d = fabs(r - cur[v]);
            out[v] = r;
            if (d > dR) dR = d;
            verts += 1;
            edges += g->in_off[v + 1] - g->in_off[v];
        }
        double *t = cur; cur = out; out = t;
        s.iterations = it + 1;
        s.final_linf = dR;
        s.vertices_processed += verts;
        s.edges_processed += edges;
        if (dR <= tol) { s.converged = 1; break; }
    }
    memcpy(ranks_out, cur, (size_t)n * sizeof(double));
    if (st) *st = s;
    free(aff); free(R); free(Rn);
    return 0;
}
