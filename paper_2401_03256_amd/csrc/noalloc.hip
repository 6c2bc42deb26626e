// Dynamic Frontier for callers that cannot allocate device memory.
//
// dfpr_pagerank_dynamic_frontier_device stages the batch (in internal ids)
// and the initial marking's source lists in a buffer the library grows with
// hipMalloc when a larger batch arrives.  The entry point here stages them
// in `scratch`, a fixed array in the library's own device memory, so that a
// call makes no allocation at all.  Each GPU the library runs on holds its
// own copy of the array until the process ends; its device address is
// looked up once per device (hipGetSymbolAddress), at the first call on that
// device, and kept.  Every call on a GPU shares that GPU's array: calls that
// overlap on one GPU (on different streams) race.  Nothing in the array
// needs clearing between calls: the batch is written in full before it is
// read, and the source lists are read only up to the counts the marking
// writes first.
#include <mutex>

#include "common.h"
#include "iter.h"

namespace dfpr {

constexpr int64_t kNoAllocMaxBatch = int64_t(1) << 20;   // batch entries a call may carry
constexpr int kMaxDevices = 64;

// the batch (4 arrays of n_del or n_ins ids) and the two source lists
static __device__ __align__(256) int32_t scratch[4 * kNoAllocMaxBatch];

static int32_t *g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device
static std::mutex g_scratch_mu;

// Device address of `scratch` on `dev`, looked up with that device current.
static int scratch_on(int dev, int32_t **out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error(DFPR_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        DFPR_HIP(hipGetDevice(&cur));
        if (cur != dev) DFPR_HIP(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) DFPR_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<int32_t *>(p);
    }
    *out = g_scratch[dev];
    return DFPR_OK;
}

}  // namespace dfpr

using namespace dfpr;

extern "C" {

int dfpr_pagerank_dynamic_frontier_device_noalloc(dfpr_graph *g, const dfpr_params *p,
                                                  int64_t n_del, const int32_t *del_src,
                                                  const int32_t *del_dst, int64_t n_ins,
                                                  const int32_t *ins_src, const int32_t *ins_dst,
                                                  const double *prev, double *ranks_out,
                                                  dfpr_stats *st)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    if (n_del < 0 || n_ins < 0) return set_error(DFPR_E_ARG, "bad batch arrays");
    if (n_del + n_ins > kNoAllocMaxBatch)
        return set_error(DFPR_E_LIMIT, "batch of " + std::to_string(n_del + n_ins) +
                                           " entries exceeds the 1048576 entries of the "
                                           "no-allocation entry point");
    dfpr_params q;
    if (p) q = *p;
    else dfpr_params_default(&q);
    // the cooperative small-frontier launch is left out of this path
    q.loop = DFPR_LOOP_LAUNCHES;
    int32_t *buf = nullptr;
    const int rc = scratch_on(g->device, &buf);
    if (rc) return rc;
    return df_device_staged(g, &q, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, prev,
                            ranks_out, st, buf);
}

}  // extern "C"
