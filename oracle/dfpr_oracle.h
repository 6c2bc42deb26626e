/*
 * CPU reference ("oracle") for Dynamic Frontier PageRank — TEST
 * INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header or
 * constant with the GPU library.
 *
 * Plain, sequential-order FP64 arithmetic written from the paper:
 *   - PageRank (Eq. 1), start from 1/n, power iteration to an L-inf
 *     tolerance (Section 3.1);
 *   - a self-loop on every vertex so that no vertex is a dead end
 *     (Section 3.1, Section 5.1.3);
 *   - a batch update = deletions then insertions (Section 3.2);
 *   - Naive-dynamic = the same iteration started from the previous ranks
 *     (Section 3.3.1);
 *   - Dynamic Frontier = initial marking, restricted rank updates and
 *     incremental marking (Section 4.1, Algorithm 1), in the synchronous
 *     form of Section 4.2 (separate input and output rank vectors);
 *   - Dynamic Traversal = the vertices reachable from the batch sources,
 *     iterated alone (Section 3.3.2).
 * Vertex loops run under OpenMP with a dynamic schedule of 2048 as in
 * Section 5.1.2; every result is independent of the thread count.
 *
 * Ranks, marks and CSRs are pinned by the tests (closed forms, dense
 * solves, the worked example of Section 4.1.2, set arithmetic).  The
 * iteration counts and work counters in oracle_stats are parity unpinned:
 * the paper prints none for any input, and a rank change near the frontier
 * tolerance can flip with the summation order.
 *
 * All functions return 0 on success and a negative code on bad input:
 *   -1 bad argument, -2 vertex id out of range, -3 out of memory.
 */
#ifndef DFPR_ORACLE_H
#define DFPR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_graph oracle_graph;

typedef struct {
    int32_t iterations;          /* iterations performed                    */
    int32_t converged;           /* 1 if Delta R <= tol was reached         */
    double final_linf;           /* Delta R of the last iteration           */
    int64_t affected_initial;    /* vertices marked by the initial marking  */
    int64_t affected_final;      /* vertices marked when the loop ended     */
    int64_t vertices_processed;  /* rank updates performed, all iterations  */
    int64_t edges_processed;     /* in-edges read, all iterations           */
} oracle_stats;

/* Build G from n vertices and m directed edges src[i] -> dst[i].
 * Duplicates are merged and a self-loop is added on every vertex. */
int oracle_load_graph(int32_t n, int64_t m, const int32_t *src,
                      const int32_t *dst, oracle_graph **out);
void oracle_free_graph(oracle_graph *g);
int oracle_graph_info(const oracle_graph *g, int32_t *n, int64_t *m);

/* Compacted CSR.  orientation 1 = out (rows are sources, entries are
 * destinations), 0 = in (rows are destinations, entries are sources).
 * offsets has n+1 entries; idx has m entries; rows are sorted ascending. */
int oracle_export_csr(const oracle_graph *g, int orientation,
                      int64_t *offsets, int32_t *idx);

/* E <- (E minus deletions) union insertions.  Self-loops are never deleted;
 * deleting an absent edge or inserting a present one changes nothing.
 * applied (nullable) receives the number of edges actually deleted and
 * actually inserted.  Any id out of range: -2 and G is left unchanged. */
int oracle_apply_batch(oracle_graph *g,
                       int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                       int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                       int64_t applied[2]);

/* Static PageRank: R = 1/n, then iterate Eq. 1 over all vertices until
 * Delta R <= tol or max_iters iterations. */
int oracle_pagerank_static(const oracle_graph *g, double alpha, double tol,
                           int32_t max_iters, double *ranks_out,
                           oracle_stats *st);

/* Naive-dynamic: as static, but starting from prev. */
int oracle_pagerank_naive_dynamic(const oracle_graph *g, double alpha,
                                  double tol, int32_t max_iters,
                                  const double *prev, double *ranks_out,
                                  oracle_stats *st);

/* Dynamic Frontier PageRank on the updated graph G^t, given the batch that
 * produced it and the previous ranks.  affected_initial / affected_final
 * (nullable, n bytes) receive the marks after the initial marking and at
 * the end.  largest_change (nullable, n doubles) receives, per vertex, the
 * largest |change of rank| over the sweeps that processed it (0 if none):
 * the quantity compared with frontier_tol, so that a caller can tell which
 * marks hinge on a comparison within rounding of the tolerance. */
int oracle_pagerank_dynamic_frontier(
    const oracle_graph *g, double alpha, double tol, double frontier_tol,
    int32_t max_iters,
    int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
    int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
    const double *prev, double *ranks_out, oracle_stats *st,
    uint8_t *affected_initial, uint8_t *affected_final, double *largest_change);

/* Initial marking on an arbitrary out-CSR (it need not hold self-loops):
 * flags[w] = 1 for every w in out(u) of each batch edge (u, v), and
 * flags[v] = 1 for each deletion (u, v), whose v was an out-neighbour of u
 * before the update.  flags (n bytes) is cleared first. */
int oracle_mark_initial_csr(int32_t n, const int64_t *out_off,
                            const int32_t *out_idx,
                            int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                            int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                            uint8_t *flags);

/* Incremental marking on an arbitrary out-CSR: next = affected, then for
 * every affected v with dr[v] > frontier_tol, next[w] = 1 for w in out(v). */
int oracle_expand_csr(int32_t n, const int64_t *out_off, const int32_t *out_idx,
                      const uint8_t *affected, const double *dr,
                      double frontier_tol, uint8_t *next);

/* Dynamic Traversal marking on an arbitrary out-CSR (Section 3.3.2):
 * flags[w] = 1 for every w reachable, in the union of the given graph and
 * the deleted edges, from the source u of any batch edge (u itself
 * included).  flags (n bytes) is cleared first. */
int oracle_mark_reachable_csr(int32_t n, const int64_t *out_off,
                              const int32_t *out_idx,
                              int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                              int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                              uint8_t *flags);

/* Dynamic Traversal PageRank on G^t: mark the reachable set, then iterate
 * Eq. 1 over it from prev until Delta R <= tol or max_iters.  affected
 * (nullable, n bytes) receives the marks. */
int oracle_pagerank_dynamic_traversal(
    const oracle_graph *g, double alpha, double tol, int32_t max_iters,
    int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
    int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
    const double *prev, double *ranks_out, oracle_stats *st, uint8_t *affected);

/* Number of OpenMP threads the oracle's parallel loops use, and a way to
 * change it (k > 0) for timing at a given thread count. */
int oracle_num_threads(void);
void oracle_set_num_threads(int k);

#ifdef __cplusplus
}
#endif

#endif
