// Internal declarations shared by the HIP sources of libdfpr.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dfpr.h"

namespace dfpr {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kBins = 7;               // in-degree classes of the pull
constexpr int kMaxGrid = 8192;         // upper bound on iteration-kernel grids
constexpr uint64_t kSentinel = ~0ull;  // batch key of an entry that changes nothing
constexpr int kCounters = 4;
// Slots the workgroups of an iteration fold their partial results into:
// ~32 workgroups share a slot at the full grid, so the per-iteration fold
// reads 256 slots instead of one partial per workgroup.
constexpr int kFoldSlots = 256;           // rows, in-edges, expanded rows, their out-edges
constexpr int kLoopChunk = 64;         // most iteration launches between two host looks

// In-degree classes.  A row of class b < 6 is reduced by a group of
// group_of(b) lanes of one wave; class 6 rows take a whole workgroup.
__host__ __device__ inline int bin_of(uint32_t deg)
{
    return deg <= 4 ? 0 : deg <= 8 ? 1 : deg <= 16 ? 2 : deg <= 32 ? 3 : deg <= 128 ? 4
           : deg <= 1024 ? 5 : 6;
}
__host__ __device__ constexpr int group_of(int bin)
{
    return bin == 0 ? 1 : bin == 1 ? 2 : bin == 2 ? 4 : bin == 3 ? 8 : bin == 4 ? 32
           : bin == 5 ? 64 : kBlock;
}

// Device control block of a graph (zeroed at creation).
struct Ctl {
    // Internal ids follow decreasing in-degree at load, so each in-degree
    // class (as the graph was loaded) is one id range: class kBins - 1 - k
    // is [cls[k], cls[k + 1]) for k < kBins, class 0 stopping where the rows
    // whose only in-entry was the self-loop begin, [cls[kBins], cls[kBins + 1]).
    // A row keeps the class of its id for the life of the graph.  Set at load.
    uint32_t cls[kBins + 2];
    uint32_t live[kBins];       // entries appended to each class list (sparse mode)
    uint32_t snap[2][kBins];    // entries iteration i processes: snap[i & 1]
    uint32_t done;              // iteration loop finished (or aborted)
    uint32_t dense;             // iterations walk the full schedule
    uint32_t force_dense;       // set during a sparse iteration: walk the full
                                // schedule from the next iteration on
    uint32_t plain_marks;       // expansions on the class lists mark with plain stores
                                // (and set force_dense) instead of appending
    uint32_t phase_end;         // the FP32 phase of the precision form is over
    int32_t phase_iters;        // iterations of the current FP32 phase
    double prev_linf;           // Delta R of the previous iteration
    double renorm_scale;        // 1 / sum of ranks (precision form)
    int32_t iterations;
    int32_t converged;
    double final_linf;
    double final_rmax;          // largest rank of the last iteration
    unsigned long long edges;   // in-edges gathered, all iterations
    unsigned long long verts;   // rank updates, all iterations
    unsigned long long xverts;  // rows that expanded (Delta r > frontier_tol)
    unsigned long long xedges;  // out-edges scanned by those expansions
    unsigned long long marked;  // vertices newly marked (sparse mode count)
    unsigned long long affected0;   // marks after the initial marking
    unsigned long long affected;    // marks when the call ended
    uint32_t err;               // an id outside [0, n) was seen
    uint32_t qn[3];             // traversal: lengths of the three level queues
    uint32_t qhn[3];            //   ... and of the three queues of heavy vertices
    uint32_t mk_light;          // initial marking: claimed sources scanned by one wave
    uint32_t mk_heavy;          //   ... and by the whole grid
    unsigned long long reach;   //   out-edges of the claimed sources
    uint32_t ntiny[2];          // batch applier: touched rows of at most 64 slots and 64 ops
    uint32_t nsmall[2];         //   ... touched rows copied to LDS
    uint32_t nbig[2];           //   ... rows whose capacity exceeds the LDS copy
    uint32_t novf[2];           //   ... rows that need a re-layout
    uint32_t max_cap[2];        //   largest row capacity
    unsigned long long top[2];  //   first free slot of each index array
    unsigned long long applied[2];  // effective deletions, insertions
    unsigned long long reach0;  // out-edges of the vertices the initial marking marked
    double ftol_used;           // frontier tolerance of the call (the adaptive rule's
                                // choice when the parameter asks for it)
    uint32_t bar[2];            // arrivals at the grid barriers of the small-frontier
                                // loop, one counter per loop phase of a call
    uint32_t loop_fail;         // a grid barrier of that loop timed out
};

// One orientation of the graph: row r holds cnt[r] sorted ids in
// idx[beg[r] .. beg[r] + cnt[r]) and owns cap[r] slots from beg[r].  Rows
// that outgrow their slots move to free space at ctl->top.
struct Csr {
    uint32_t *beg = nullptr;    // n
    uint32_t *cnt = nullptr;    // n live counts
    uint32_t *cap = nullptr;    // n capacities
    int32_t *idx = nullptr;     // `slots` entries
    uint64_t slots = 0;
    uint32_t max_cap = 0;       // largest row capacity (host copy)
};

struct IterBufs {
    // kFoldSlots slots each; workgroup w of an iteration folds its results
    // into slot w mod kFoldSlots with atomics, the per-iteration fold reads
    // and clears every slot
    double *dr_part = nullptr;                // L-inf of Delta r (atomic max on the bits)
    double *rmax_part = nullptr;              // largest rank (atomic max on the bits)
    unsigned long long *cnt_part = nullptr;   // counters (kCounters per slot)
};

// Host-side profile of the iteration kernel (see dfpr_profile in dfpr.h).
struct Profile {
    int enabled = 0;
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
    int64_t rows = 0, edges = 0, exp_rows = 0, exp_edges = 0, marked = 0;
};

struct ApplyBufs {
    uint64_t cap = 0;               // batch entries the buffers hold
    uint64_t *keys[2][2] = {};      // [orientation][ping-pong]
    uint32_t *tiny_list[2] = {};    // op index where each touched row starts, by row size
    uint32_t *small_list[2] = {};
    uint32_t *big_list[2] = {};
    uint32_t *ovf_list[2] = {};
    int32_t *ovf_need[2] = {};      // capacity an overflowed row needs
    unsigned long long *part = nullptr;  // per-workgroup applied counts (deletions, insertions)
    int32_t *slab = nullptr;        // row copies of big rows
    uint64_t slab_ints = 0;
    uint64_t slab_stride = 0;
    int32_t *batch_dev = nullptr;   // batch in internal ids (4 arrays) + marking lists
    uint64_t batch_cap = 0;
    int32_t *batch_host = nullptr;  // pinned staging of a host batch (4 arrays)
    uint64_t batch_host_cap = 0;
};

}  // namespace dfpr

// Vertices are renumbered at load: internal ids follow decreasing in-degree
// (ties by the caller's id), so that the rows of one in-degree class form a
// contiguous id range and high-degree sources share cache lines.  Every id,
// rank and flag that crosses the C-ABI is in the caller's numbering.
struct dfpr_graph {
    int32_t n = 0;
    int64_t m = 0;                    // live edges, self-loops included
    int32_t *ext2int = nullptr;       // device: caller id -> internal id
    int32_t *int2ext = nullptr;       // device: internal id -> caller id
    std::vector<int32_t> ext2int_h;   // host copies of the two maps
    std::vector<int32_t> int2ext_h;
    double *Rx = nullptr;             // n ranks in the caller's numbering (staging)
    dfpr::Csr csr[2];                 // [0] = in (rows = dst), [1] = out (rows = src)
    double *R[2] = {};                // rank double buffer
    double *C[2] = {};                // contribution R[v] / |out(v)|
    int cur = 0;                      // buffer holding the resident ranks
    uint32_t *stamp = nullptr;        // iteration a vertex was marked (see rank.hip)
    uint32_t *xstamp = nullptr;       // call in which a vertex expanded
    uint32_t *mstamp = nullptr;       // stamps of the marking-only calls (their own,
    uint32_t *mxstamp = nullptr;      //   so those calls keep the last update's marks)
    uint32_t next_base = 1;           // stamp base of the next call
    uint32_t last_base = 0;           // stamp base and iterations of the last
    int32_t last_iters = -1;          //   Dynamic Frontier or Traversal call
    int32_t *bins = nullptr;          // kBins appended lists of n entries (sparse mode)
    int32_t *bfs_q = nullptr;         // traversal: 3 light + 3 heavy level queues, n each
    // id ranges of the in-degree classes at load (host copy of Ctl::cls):
    // the full schedule walks them in place of a list of all vertices
    uint32_t cls[dfpr::kBins + 2] = {};
    dfpr::Ctl *ctl = nullptr;         // device
    dfpr::Ctl *ctl_host = nullptr;    // pinned, coherent mirror (written by the kernels
                                      // that end a loop step, or copied)
    dfpr::IterBufs it;
    dfpr::ApplyBufs ap;
    float *C32[2] = {};               // FP32 contributions (precision form)
    double *scratch_sum = nullptr;    // FP64 reduction scratch
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;     // a call's device time
    hipEvent_t ev_mid = nullptr;                 // its first iteration's start
    hipEvent_t ev_a0 = nullptr, ev_a1 = nullptr; // the last batch application
    float last_apply_ms = 0.f;
    hipEvent_t evk[4 * dfpr::kLoopChunk] = {};   // around each iteration launch (profiling),
                                                 // per chunk slot
    hipEvent_t evc[2] = {};                      // completion of the chunk in each slot
    dfpr::Profile prof;
    int64_t prof_base[5] = {0, 0, 0, 0, 0};   // counters already added to prof
    int32_t refine_sweeps = 0;        // FP64 iterations after the FP32 phase
    int32_t loop_iters = 0;           // iterations the small-frontier loop ran
    int busy = 0;
    int device = 0;                   // the HIP device the graph lives on
    int grid = 1024;                  // iteration-kernel workgroups
    int grid_wide = 1024;             //   ... of the wide full-sweep kernel
    int grid_wide_df = 1024;          //   ... of the wide Dynamic Frontier kernel
    int coop = 0;                     // the device takes cooperative launches
    uint32_t sparse_limit = 0;        // frontier size that switches to the full schedule
};

namespace dfpr {

int set_error(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define DFPR_HIP(call)                                          \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return dfpr::hip_fail(e_, #call); \
    } while (0)

// Return a library status other than DFPR_OK to the caller.
#define DFPR_CHECK_RC(call)             \
    do {                                \
        const int rc_ = (call);         \
        if (rc_ != 0) return rc_;       \
    } while (0)

// batch applier (apply.hip)
int apply_batch_impl(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                     int64_t n_ins, const int32_t *is, const int32_t *id, int on_device,
                     int64_t applied[2]);
int stage_batch(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                int64_t n_ins, const int32_t *is, const int32_t *id, int on_device,
                const int32_t **dds, const int32_t **ddd, const int32_t **dis,
                const int32_t **did);
// The same for device arrays, into a caller-chosen buffer of at least
// 2 (n_del + n_ins) ints (no allocation).
int stage_batch_into(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                     int64_t n_ins, const int32_t *is, const int32_t *id, int32_t *buf,
                     const int32_t **dds, const int32_t **ddd, const int32_t **dis,
                     const int32_t **did);
int check_ids_host(int32_t n, int64_t len, const int32_t *a, const int32_t *b);

// renumbering at the boundary (graph.hip); enqueued on g->stream
int map_ids(dfpr_graph *g, const int32_t *in, int32_t *out, int64_t len);
int map_ids4(dfpr_graph *g, const int32_t *const in[4], const int64_t len[4], int32_t *out);
int ranks_to_caller(const dfpr_graph *g, const double *Rint, double *out, int out_dev);
int ranks_from_caller(const dfpr_graph *g, const double *in, int in_dev, double *Rint);

// device helpers (rank.hip)
int64_t apply_slab_bytes(const dfpr_graph *g);
int launch_fill_u32(dfpr_graph *g, uint32_t *p, uint64_t len, uint32_t value);
// Enqueue the copy of the control block to its host copy (g->ctl_host) on
// the graph's stream; the host reads it after synchronising the stream.
int ctl_to_host(dfpr_graph *g);

}  // namespace dfpr
