/*
 * dfpr.h — Dynamic Frontier PageRank on one AMD Instinct MI355X (gfx950).
 *
 * C-ABI of libdfpr.so.  Plain pointers and sizes only.  Every call returns a
 * status code (DFPR_OK = 0, negative on error); on error a message is
 * available from dfpr_last_error() (thread-local) and, unless stated
 * otherwise, the graph is left as it was before the call.
 *
 * The method (Sahu, "An Incrementally Expanding Approach for Updating
 * PageRank on Dynamic Graphs"):
 *   - PageRank of v:  R[v] = alpha * sum_{u in in(v)} R[u]/|out(u)| + (1-alpha)/n
 *     (Eq. 1), solved by power iteration from R = 1/n until the L-inf change
 *     of an iteration is <= tol (Section 3.1);
 *   - every vertex carries a self-loop, so there are no dead ends
 *     (Section 3.1, Section 5.1.3);
 *   - a batch update is a set of deletions and a set of insertions of
 *     edges; vertices are never added or removed (Section 3.2, 5.1.4);
 *   - Naive-dynamic restarts the iteration from the previous ranks
 *     (Section 3.3.1);
 *   - Dynamic Frontier marks the out-neighbours (before and after the update)
 *     of the source of every changed edge, recomputes only marked vertices,
 *     and marks the out-neighbours of any vertex whose rank moved by more
 *     than frontier_tol, until the L-inf change is <= tol (Section 4.1,
 *     Algorithm 1).
 * This library runs the synchronous form of Section 4.2: each iteration
 * reads one rank vector and writes another; vertices marked during an
 * iteration are processed from the next one; marks are never cleared within
 * one update.  Ranks are FP64 and vertex ids int32 (Section 5.1.2).
 *
 * Memory.  The library owns all device memory of a graph: the in-edge CSR
 * (for the pull of Eq. 1) and the out-edge CSR (for marking and |out(u)|),
 * both with per-row slack so a batch is merged in place, the two rank
 * vectors and the work lists.  Pointers documented as "host" are ordinary
 * host memory, borrowed for the duration of the call.  Pointers documented
 * as "device" are device memory of the current HIP device, borrowed for the
 * call and accessed on the graph's stream.
 *
 * Threading.  One writer per graph (Section 3.2): calls on one graph must
 * not overlap.  Different graphs may be used from different threads.
 */
#ifndef DFPR_H
#define DFPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DFPR_OK 0
#define DFPR_E_ARG (-1)     /* bad argument (null pointer, negative size, ...) */
#define DFPR_E_RANGE (-2)   /* a vertex id is outside [0, n)                   */
#define DFPR_E_NOMEM (-3)   /* device or host allocation failed                */
#define DFPR_E_DEVICE (-4)  /* a HIP call failed                               */
#define DFPR_E_BUSY (-5)    /* the graph is in use by another call             */
#define DFPR_E_LIMIT (-6)   /* graph too large for 32-bit edge offsets         */

/* precision forms */
#define DFPR_FP64 0         /* ranks and contributions in FP64 (the method)   */
#define DFPR_FP32_KAHAN 1   /* FP32 contributions, compensated FP32 row sums,
                               FP64 L-inf, renormalisation and final FP64
                               sweeps (see dfpr_pagerank_dynamic_frontier)    */

/* iteration forms (dfpr_params.mode) */
#define DFPR_SYNC 0         /* separate input and output rank vectors          */
#define DFPR_ASYNC 1        /* one rank vector updated in place                 */

/* dfpr_params.frontier_tol: choose it per call (see dfpr_params) */
#define DFPR_FTOL_ADAPTIVE (-1.0)

/* iteration drivers (dfpr_params.loop) */
#define DFPR_LOOP_LAUNCHES 0 /* one launch pair per iteration                   */
#define DFPR_LOOP_DEVICE 1   /* small frontiers iterate inside one launch       */

typedef struct dfpr_graph dfpr_graph;

typedef struct {
    double alpha;          /* damping factor; default 0.85 (Section 5.1.2)      */
    double tol;            /* iteration tolerance tau on the L-inf change;
                              default 1e-10 (Section 5.1.2)                     */
    double frontier_tol;   /* frontier tolerance tau_f; a vertex whose rank
                              changes by MORE than this marks its out-
                              neighbours; default tol/1e5 (Section 4.3).  A
                              negative value (DFPR_FTOL_ADAPTIVE) lets each
                              Dynamic Frontier call choose tol/10^k, k = 1..5,
                              from the mean out-degree g of the vertices its
                              initial marking marked: k = 1 for g <= 8, 2 for
                              g <= 16, 3 for g <= 32, 4 for g <= 64, else 5
                              (Section 5.2.4: the suitable tau_f depends on
                              the batch; the choice is reported in
                              dfpr_stats.frontier_tol_used)                   */
    int32_t max_iters;     /* iteration cap; default 500 (Section 5.1.2)       */
    int32_t precision;     /* DFPR_FP64 (default) or DFPR_FP32_KAHAN           */
    int32_t mode;          /* DFPR_SYNC (default): every iteration reads the
                              previous iteration's ranks (Section 4.2's
                              synchronous form); DFPR_ASYNC: one rank vector
                              updated in place, so an iteration may read ranks
                              written earlier in the same iteration (the
                              asynchronous form, Section 4.2).  ASYNC results
                              are not bitwise reproducible; it applies to the
                              FP64 iterations (not to the FP32 phase) and is
                              ignored by the serving calls.                    */
    int32_t loop;          /* DFPR_LOOP_LAUNCHES (default): every iteration
                              is its own launch pair (pull, then fold);
                              DFPR_LOOP_DEVICE: while a Dynamic Frontier
                              call's frontier is small, its iterations run
                              inside one cooperative launch (Algorithm 1's
                              loop on the device, a grid barrier between the
                              pull and the fold).  Results are bitwise the
                              same either way; on MI355X the launch pairs are
                              as fast or faster at every frontier measured. */
} dfpr_params;

typedef struct {
    int32_t iterations;         /* iterations performed (FP64 iterations in
                                   the FP32 form count separately below)      */
    int32_t converged;          /* 1 if the L-inf change reached <= tol;
                                   reaching max_iters is not an error         */
    int32_t refine_sweeps;      /* FP64 iterations after the FP32 phase       */
    int32_t loop_iterations;    /* iterations run inside the small-frontier
                                   loop (see dfpr_params.loop)                */
    double final_linf;          /* L-inf change of the last iteration          */
    double ms_device;           /* device time of the call (HIP events)        */
    int64_t affected_initial;   /* vertices marked by the initial marking      */
    int64_t affected_final;     /* vertices marked when the loop ended         */
    int64_t vertices_processed; /* rank updates, summed over iterations        */
    int64_t edges_processed;    /* in-edges gathered, summed over iterations   */
    double ms_mark;             /* part of ms_device before the first
                                   iteration: batch staging, starting ranks
                                   and the initial marking
                                   (Dynamic Frontier) or the reachability
                                   search (Dynamic Traversal)                 */
    double ms_iter;             /* the rest of ms_device: iterations (FP32
                                   phase, renormalisation, refinement) and the
                                   closing pass over the marks                 */
    double ms_apply;            /* device time of the last dfpr_apply_batch or
                                   dfpr_apply_batch_device on this graph (0 if
                                   none, or if it was empty); not in ms_device */
    double frontier_tol_used;   /* frontier tolerance of a Dynamic Frontier
                                   call (the adaptive choice, if asked for);
                                   0 for the other methods                    */
} dfpr_stats;

/* Defaults of Section 5.1.2 and Section 4.3. */
void dfpr_params_default(dfpr_params *p);

/* Build a graph of n vertices (1 <= n < 2^31) from m directed edges
 * src[i] -> dst[i] (host arrays).  Repeated edges count once and a
 * self-loop is added to every vertex (Section 3.1).  The ranks held by the
 * graph start at 1/n.  Rows get slack of max(2, deg/8) entries.
 * Internally the library renumbers the vertices by decreasing in-degree;
 * every id, rank and flag passed to or returned by any call stays in the
 * caller's numbering.
 * *out receives a handle owned by the library (free with dfpr_free_graph).
 * Errors: DFPR_E_ARG, DFPR_E_RANGE (id outside [0, n)), DFPR_E_NOMEM,
 * DFPR_E_LIMIT (more than 2^32 - 1 edge slots). */
int dfpr_load_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    dfpr_graph **out);

/* Free the graph and all its device memory.  NULL is ignored. */
void dfpr_free_graph(dfpr_graph *g);

/* Make the graph issue its work on this HIP stream (hipStream_t passed as
 * void*); NULL selects the graph's own stream (the default).  The stream
 * must stay valid while the graph uses it. */
int dfpr_set_stream(dfpr_graph *g, void *hip_stream);

/* Number of vertices and of edges (self-loops included) of G. */
int dfpr_graph_info(const dfpr_graph *g, int32_t *n, int64_t *m);

/* Apply one batch update (Section 3.2): E <- (E minus deletions) union
 * insertions, on both CSRs, on the device.  Host arrays.  Deletions are
 * applied before insertions; deleting a self-loop or an absent edge and
 * inserting a present edge change nothing; repeats count once.
 * applied (host, nullable, 2 entries) receives the number of edges
 * actually deleted and actually inserted.  Any id outside [0, n): the
 * whole batch is rejected with DFPR_E_RANGE and G is unchanged. */
int dfpr_apply_batch(dfpr_graph *g,
                     int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                     int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                     int64_t applied[2]);

/* As dfpr_apply_batch, with the four id arrays in device memory.
 * applied stays a host pointer (nullable). */
int dfpr_apply_batch_device(dfpr_graph *g,
                            int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                            int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                            int64_t applied[2]);

/* Static PageRank (Section 3.1): R = 1/n, then iterate Eq. 1 over all
 * vertices until the L-inf change is <= p->tol or p->max_iters iterations.
 * p NULL selects the defaults.  ranks_out (host, n doubles, nullable)
 * receives the ranks, which also become the graph's resident ranks.
 * st (host, nullable) receives statistics. */
int dfpr_pagerank_static(dfpr_graph *g, const dfpr_params *p, double *ranks_out,
                         dfpr_stats *st);

/* Naive-dynamic PageRank (Section 3.3.1): as static, but starting from
 * prev (host, n doubles) or, if prev is NULL, from the graph's resident
 * ranks.  ranks_out (host, nullable) may alias prev. */
int dfpr_pagerank_naive_dynamic(dfpr_graph *g, const dfpr_params *p,
                                const double *prev, double *ranks_out,
                                dfpr_stats *st);

/* Dynamic Frontier PageRank (Algorithm 1) on the current graph G^t.  The
 * batch (host arrays) is the one that produced G^t from G^{t-1}, i.e. the
 * one last given to dfpr_apply_batch.  prev (host, nullable: resident
 * ranks) holds R^{t-1}; ranks_out (host, nullable) receives R^t, which also
 * becomes the resident ranks.  Ids are checked as in dfpr_apply_batch.
 *
 * With p->precision == DFPR_FP32_KAHAN the marked vertices are first
 * iterated with FP32 contributions and compensated FP32 row sums (Delta r
 * and the L-inf test in FP64) until the change stalls at FP32 resolution;
 * the ranks are then renormalised to sum 1 in FP64 and the FP64 iteration
 * continues over the marked vertices until the L-inf change is <= tol. */
int dfpr_pagerank_dynamic_frontier(dfpr_graph *g, const dfpr_params *p,
                                   int64_t n_del, const int32_t *del_src,
                                   const int32_t *del_dst, int64_t n_ins,
                                   const int32_t *ins_src, const int32_t *ins_dst,
                                   const double *prev, double *ranks_out,
                                   dfpr_stats *st);

/* As dfpr_pagerank_dynamic_frontier with the batch arrays, prev and
 * ranks_out in device memory (prev and ranks_out nullable as above).  The
 * ids are checked on the device: an id outside [0, n) ends the call with
 * DFPR_E_RANGE before any iteration, the resident ranks then being prev if
 * given, else unchanged. */
int dfpr_pagerank_dynamic_frontier_device(dfpr_graph *g, const dfpr_params *p,
                                          int64_t n_del, const int32_t *del_src,
                                          const int32_t *del_dst, int64_t n_ins,
                                          const int32_t *ins_src,
                                          const int32_t *ins_dst, const double *prev,
                                          double *ranks_out, dfpr_stats *st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * dfpr_pagerank_dynamic_frontier_device, but the batch is staged in a
 * fixed array the library holds on each GPU (16 MiB, kept until the process
 * ends) instead of a buffer it grows on demand, so the call makes no
 * allocation.  n_del + n_ins may be at most 1048576 (DFPR_E_LIMIT beyond,
 * nothing changed).  Every call on a GPU shares that array: calls that
 * overlap on one GPU race.  Iterations run as launch pairs whatever
 * p->loop asks for. */
int dfpr_pagerank_dynamic_frontier_device_noalloc(dfpr_graph *g, const dfpr_params *p,
                                                  int64_t n_del, const int32_t *del_src,
                                                  const int32_t *del_dst, int64_t n_ins,
                                                  const int32_t *ins_src,
                                                  const int32_t *ins_dst, const double *prev,
                                                  double *ranks_out, dfpr_stats *st);

/* Dynamic Traversal PageRank (Section 3.3.2), a comparator: every vertex
 * reachable from the source of a batch edge in G^{t-1} or in G^t is
 * updated, from prev (NULL = the resident ranks), until Delta R <= tol or
 * max_iters; no vertex joins during the iterations.  G^t must already hold
 * the batch (dfpr_apply_batch).  Arguments, errors and outputs as
 * dfpr_pagerank_dynamic_frontier (host arrays); frontier_tol and precision
 * are ignored (FP64).  st->affected_initial = affected_final = the
 * reachable count. */
int dfpr_pagerank_dynamic_traversal(dfpr_graph *g, const dfpr_params *p, int64_t n_del,
                                    const int32_t *del_src, const int32_t *del_dst,
                                    int64_t n_ins, const int32_t *ins_src,
                                    const int32_t *ins_dst, const double *prev,
                                    double *ranks_out, dfpr_stats *st);

/* The reachable set of Dynamic Traversal alone: flags_out[v] = 1 (n bytes,
 * caller's numbering) for every v reachable from a batch source along G^t's
 * out-edges and the batch's deleted edges, the sources included.  Host
 * arrays; DFPR_E_RANGE for an id outside [0, n). */
int dfpr_mark_reachable(dfpr_graph *g, int64_t n_del, const int32_t *del_src,
                        const int32_t *del_dst, int64_t n_ins, const int32_t *ins_src,
                        const int32_t *ins_dst, uint8_t *flags_out);

/* Initial marking only (Section 4.1.1, first rule): flags_out (host, n
 * bytes) receives 1 for every w in G^t.out(u) of each batch edge (u, v) and
 * for the v of each deletion, 0 elsewhere.  Ranks are not touched. */
int dfpr_mark_affected(dfpr_graph *g,
                       int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                       int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                       uint8_t *flags_out);

/* Marks held when the last Dynamic Frontier or Dynamic Traversal call on
 * this graph ended: flags_out[v] = 1 (host, n bytes, caller's numbering)
 * for every vertex it marked affected, those marked in its last iteration
 * included; all 0 before the first such call.  dfpr_mark_affected and
 * dfpr_mark_reachable keep their marks apart and leave these unchanged. */
int dfpr_get_affected(const dfpr_graph *g, uint8_t *flags_out);

/* Copy the resident ranks out (host or device pointer, n doubles). */
int dfpr_get_ranks(const dfpr_graph *g, double *ranks, int on_device);

/* Replace the resident ranks (host or device pointer, n doubles, in the
 * caller's vertex numbering); NULL restores the uniform start 1/n.
 * DFPR_E_BUSY while another call uses the graph. */
int dfpr_set_ranks(dfpr_graph *g, const double *ranks, int on_device);

/* Compacted CSR of G (host arrays): out_orientation 1 gives rows = sources,
 * entries = destinations; 0 gives rows = destinations, entries = sources.
 * offsets has n+1 entries, idx has m entries (dfpr_graph_info); each row is
 * sorted ascending. */
int dfpr_export_csr(const dfpr_graph *g, int out_orientation, int64_t *offsets,
                    int32_t *idx);

/* Profile of the iteration kernel (the pull, Delta r, L-inf and expansion
 * of one iteration), summed over every call made while profiling is on.
 * ms is measured with HIP events recorded on the graph's stream right
 * before and after each iteration-kernel launch (timing-only events, with
 * no system-scope fence).  bytes is the algorithmic traffic of those
 * launches: per processed row 40 bytes (list entry, row start and length,
 * R[v], |out(v)|, the two written values; 36 with an FP32 contribution)
 * plus 8 in Dynamic Frontier (its mark and expansion stamp); per in-edge
 * 12 bytes (index and gathered FP64 contribution; 8 in FP32); per
 * expanding row 8 bytes (out-row start and length) plus 8 per out-edge it
 * scans (index and the target's mark). */
typedef struct {
    int64_t launches;        /* iteration-kernel launches                  */
    double ms;               /* their device time                          */
    double bytes;            /* their algorithmic bytes                    */
    int64_t rows;            /* rank updates                               */
    int64_t edges;           /* in-edges gathered                          */
    int64_t expanded_rows;   /* rows whose change exceeded frontier_tol     */
    int64_t expanded_edges;  /* out-edges those rows scanned               */
    int64_t marked;          /* vertices newly marked by expansion in sparse
                                iterations (dense ones mark with plain stores
                                and do not count)                           */
} dfpr_profile;

/* Zero the profile and switch profiling on (enable != 0) or off. */
int dfpr_profile_reset(dfpr_graph *g, int enable);

/* Read the profile accumulated since the last dfpr_profile_reset. */
int dfpr_profile_read(const dfpr_graph *g, dfpr_profile *out);

/* ---- serving form --------------------------------------------------------
 * A server keeps several graphs resident and serves update requests
 * (graph, batch) that arrive over time, by continuous batching: a request is
 * admitted into one of max_slots slots when a slot is free, its graph has no
 * update in flight (one writer per graph, Section 3.2) and the HBM budget
 * covers the resident graphs (graph store, ranks, marks, schedule and the
 * applier's copies of long rows, estimated when the graph is added) plus
 * the scratch of the requests in flight (96 bytes per batch entry).  Admission applies the batch (as
 * dfpr_apply_batch) and runs the initial marking; then every step runs one
 * Dynamic Frontier iteration of every admitted request in one coalesced
 * launch.  Steps run in chunks between two looks by the host (kept to about
 * a millisecond while requests wait), and a finished request frees its
 * slot at the end of its chunk; admissions run on a second stream while a
 * chunk is on the device.  A request's
 * result equals that of dfpr_apply_batch followed by
 * dfpr_pagerank_dynamic_frontier with the graph's parameters, whatever else
 * is in flight.  The server borrows its graphs; they must stay alive and
 * must not be used by other calls during dfpr_server_run. */

typedef struct dfpr_server dfpr_server;

typedef struct {
    int64_t requests, completed, failed;
    double wall_ms;            /* start of dfpr_server_run to the last completion   */
    double updates_per_s;      /* completed requests / wall time                    */
    double latency_p50_ms, latency_p99_ms, latency_mean_ms;   /* arrival to ranks ready */
    double queue_p50_ms, queue_p99_ms;                        /* arrival to admission   */
    int32_t max_active;        /* most requests in flight at once                   */
    int32_t steps;             /* coalesced iteration launches                      */
    int64_t peak_bytes;        /* largest resident + in-flight budget use           */
} dfpr_server_stats;

typedef struct {
    int32_t graph_id;
    int32_t status;            /* DFPR_OK, or the error that rejected the request   */
    int32_t iterations, refine_sweeps, converged, reserved;
    double arrival_ms, admit_ms, done_ms;   /* relative to the start of the run      */
    int64_t applied[2];        /* effective deletions and insertions                */
    int64_t edges_processed, affected;
    double final_linf;
} dfpr_request_result;

/* max_slots in [1, 8]; hbm_budget_bytes > 0.  *out receives a handle owned
 * by the library (free with dfpr_server_free).  DFPR_E_ARG, DFPR_E_NOMEM,
 * DFPR_E_DEVICE. */
int dfpr_server_create(int32_t max_slots, int64_t hbm_budget_bytes, dfpr_server **out);
void dfpr_server_free(dfpr_server *s);

/* Requests on graphs of at least large_edges edges (self-loops included)
 * run in the server's large lane: one at a time, in arrival order, on a
 * stream of their own; all other requests share coalesced steps in the
 * small lane.  Default 2^25 (a graph whose full sweep fills an MI355X).
 * Applies to the graphs already added and to later ones.  DFPR_E_ARG for
 * large_edges < 1. */
int dfpr_server_set_large_edges(dfpr_server *s, int64_t large_edges);

/* Add a resident graph (parameters p, NULL = defaults; p->precision picks
 * FP64 or the FP32 form for its updates).  DFPR_E_NOMEM if the resident
 * graphs would exceed the budget.  *graph_id receives its index. */
int dfpr_server_add_graph(dfpr_server *s, dfpr_graph *g, const dfpr_params *p,
                          int32_t *graph_id);

/* Queue a request (host arrays, copied) arriving arrival_ms >= 0 after the
 * start of dfpr_server_run.  *request_id receives its index.  DFPR_E_ARG for
 * an unknown graph or bad arrays, DFPR_E_NOMEM if the request alone can
 * never fit the budget. */
int dfpr_server_submit(dfpr_server *s, int32_t graph_id, double arrival_ms,
                       int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                       int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                       int64_t *request_id);

/* Serve every request queued since the last run, admitting each no earlier
 * than its arrival time, and return when all are done.  A request whose
 * batch holds an id outside [0, n) fails (status DFPR_E_RANGE) without
 * changing its graph.  DFPR_E_BUSY if a graph is in use by another call;
 * device errors end the run with DFPR_E_DEVICE: the requests then in flight
 * fail with that status and the ranks of their graphs are undefined. */
int dfpr_server_run(dfpr_server *s, dfpr_server_stats *st);

/* Outcome of one request after dfpr_server_run. */
int dfpr_server_result(const dfpr_server *s, int64_t request_id, dfpr_request_result *out);

/* Message for the last non-OK status returned on this thread. */
const char *dfpr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
