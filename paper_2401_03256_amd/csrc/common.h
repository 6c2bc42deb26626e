// Internal declarations shared by the HIP sources of libdfpr.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "dfpr.h"

namespace dfpr {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr int kBins = 6;             // in-degree classes of the pull
constexpr int kMaxGrid = 4096;       // upper bound on iteration-kernel grids
constexpr uint64_t kSentinel = ~0ull;  // batch key of an entry that changes nothing

// In-degree classes.  A row of class b is reduced by a group of
// kGroup[b] lanes; class 5 rows take a whole workgroup.
__host__ __device__ inline int bin_of(uint32_t deg)
{
    return deg <= 4 ? 0 : deg <= 8 ? 1 : deg <= 16 ? 2 : deg <= 32 ? 3 : deg <= 1024 ? 4 : 5;
}

// Device control block of a graph (zeroed at creation).
struct Ctl {
    uint32_t live[kBins];       // entries appended to each class list
    uint32_t snap[2][kBins];    // entries iteration i processes: snap[i & 1]
    uint32_t ticket;            // workgroups finished in the current iteration
    uint32_t done;              // iteration loop finished (or aborted)
    int32_t iterations;
    int32_t converged;
    double final_linf;
    unsigned long long edges;   // in-edges gathered, all iterations
    unsigned long long verts;   // rank updates, all iterations
    uint32_t err;               // an id outside [0, n) was seen
    uint32_t nsmall[2];         // batch applier: touched rows per orientation
    uint32_t nbig[2];           //   ... rows whose capacity exceeds the LDS copy
    uint32_t novf[2];           //   ... rows whose slack was too small
    uint32_t pad0;
    unsigned long long applied[2];  // effective deletions, insertions
    unsigned long long affected0;   // marks after the initial marking
};

// One orientation of the graph: row r holds cnt[r] sorted ids in
// idx[beg[r] .. beg[r] + cnt[r]) and owns the slots up to beg[r+1].
struct Csr {
    uint32_t *beg = nullptr;    // n + 1 capacity offsets
    uint32_t *cnt = nullptr;    // n live counts
    int32_t *idx = nullptr;     // beg[n] slots
    uint64_t slots = 0;
    uint32_t max_cap = 0;       // largest row capacity
};

struct IterBufs {
    double *dr_part = nullptr;                 // per-workgroup L-inf partials
    unsigned long long *edges_part = nullptr;  // per-workgroup edge counts
    unsigned long long *verts_part = nullptr;
};

struct ApplyBufs {
    uint64_t cap = 0;               // batch entries the buffers hold
    uint64_t *keys[2][2] = {};      // [orientation][ping-pong]
    uint32_t *small_list[2] = {};   // op-start index of touched rows
    uint32_t *big_list[2] = {};
    uint32_t *ovf_list[2] = {};
    int32_t *ovf_need[2] = {};      // capacity an overflowed row needs
    int32_t *slab = nullptr;        // row copies of big rows
    uint64_t slab_ints = 0;
    int32_t *batch_dev = nullptr;   // staging for host batches (4 arrays)
    uint64_t batch_cap = 0;
};

}  // namespace dfpr

struct dfpr_graph {
    int32_t n = 0;
    int64_t m = 0;                    // live edges, self-loops included
    dfpr::Csr csr[2];                 // [0] = in (rows = dst), [1] = out (rows = src)
    double *R[2] = {};                // rank double buffer
    double *C[2] = {};                // contribution R[v] / |out(v)|
    int cur = 0;                      // buffer holding the resident ranks
    uint8_t *flags = nullptr;         // affected marks (n rounded up to 4)
    int32_t *bins = nullptr;          // kBins lists of n entries each
    dfpr::Ctl *ctl = nullptr;         // device
    dfpr::Ctl *ctl_host = nullptr;    // pinned mirror
    dfpr::IterBufs it;
    dfpr::ApplyBufs ap;
    float *C32[2] = {};               // FP32 contributions (precision form)
    double *scratch_sum = nullptr;    // FP64 reduction scratch
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int busy = 0;
    int grid = 1024;                  // iteration-kernel workgroups
};

namespace dfpr {

int set_error(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define DFPR_HIP(call)                                      \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return dfpr::hip_fail(e_, #call); \
    } while (0)

// batch applier (apply.hip)
int apply_batch_impl(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                     int64_t n_ins, const int32_t *is, const int32_t *id, int on_device,
                     int64_t applied[2]);
int stage_batch(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                int64_t n_ins, const int32_t *is, const int32_t *id,
                const int32_t **dds, const int32_t **ddd, const int32_t **dis,
                const int32_t **did);
int check_ids_host(int32_t n, int64_t len, const int32_t *a, const int32_t *b);

// device helpers (rank.hip)
int launch_fill_u8(dfpr_graph *g, uint8_t *p, uint64_t len);
int recompute_contrib(dfpr_graph *g);

}  // namespace dfpr
