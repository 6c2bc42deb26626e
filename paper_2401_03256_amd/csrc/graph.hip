// Graph store: loading, freeing, export, resident ranks, errors.
//
// A graph lives in device memory as two CSRs with per-row slack:
//   csr[0] (in-edges)  : row v lists G.in(v), used by the pull of Eq. 1;
//   csr[1] (out-edges) : row u lists G.out(u); its live count is |out(u)|.
// Loading (not timed by the paper, Section 5.1.5) is done on the host with
// counting sorts and then copied up once.  Vertices get internal ids in
// order of decreasing in-degree (stable in the caller's ids); the maps
// between the two numberings are applied wherever ids or per-vertex values
// cross the C-ABI.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"

namespace dfpr {

// Iteration-kernel workgroups per CU.  The kernel fits five waves per SIMD,
// so most of the grid waits for a free slot; many small workgroups even
// out the uneven rows (32 per CU measured best on R-MAT scale 22, 5% over 8).
#ifndef DFPR_GRID_PER_CU
#define DFPR_GRID_PER_CU 32
#endif
constexpr int kGridPerCU = DFPR_GRID_PER_CU;
// Workgroups per CU of the wide full-schedule kernels: 12-wave sweeps (two
// resident per CU; 11 beat 8 and 16) and 8-wave Dynamic Frontier
// iterations (three resident per CU).
#ifndef DFPR_WIDE_GRID_PER_CU
#define DFPR_WIDE_GRID_PER_CU 11
#endif
#ifndef DFPR_WIDE_DF_GRID_PER_CU
#define DFPR_WIDE_DF_GRID_PER_CU 16
#endif
constexpr int kWideGridPerCU = DFPR_WIDE_GRID_PER_CU;
constexpr int kWideDfGridPerCU = DFPR_WIDE_DF_GRID_PER_CU;

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return set_error(e == hipErrorOutOfMemory ? DFPR_E_NOMEM : DFPR_E_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

int check_ids_host(int32_t n, int64_t len, const int32_t *a, const int32_t *b)
{
    for (int64_t i = 0; i < len; i++)
        if (a[i] < 0 || a[i] >= n || b[i] < 0 || b[i] >= n)
            return set_error(DFPR_E_RANGE, "vertex id outside [0, n) at batch entry " +
                                                std::to_string(i));
    return DFPR_OK;
}

// Slack given to a row of `deg` live entries.
static inline uint64_t row_capacity(uint64_t deg)
{
    return deg + std::max<uint64_t>(2, deg / 8);
}

// Free slots kept after the packed rows for rows that outgrow their slack.
static inline uint64_t spill_reserve(uint64_t packed)
{
    return std::max<uint64_t>(packed / 16, 1 << 16);
}

// Build one padded CSR on the host from sorted rows (off/idx, compacted)
// and upload it.  *top receives the first free slot.
static int upload_csr(Csr &c, int32_t n, const std::vector<uint64_t> &off,
                      const std::vector<int32_t> &idx, uint32_t *top)
{
    std::vector<uint32_t> beg(n), cnt(n), cap(n);
    uint64_t pos = 0;
    uint32_t max_cap = 0;
    for (int32_t r = 0; r < n; r++) {
        uint64_t d = off[r + 1] - off[r];
        uint64_t cp = row_capacity(d);
        beg[r] = (uint32_t)pos;
        cnt[r] = (uint32_t)d;
        cap[r] = (uint32_t)cp;
        max_cap = std::max<uint32_t>(max_cap, (uint32_t)cp);
        pos += cp;
    }
    const uint64_t slots = pos + spill_reserve(pos);
    if (slots > 0xFFFFFFFFull)
        return set_error(DFPR_E_LIMIT, "graph needs more than 2^32-1 edge slots");
    std::vector<int32_t> packed(pos, -1);
    for (int32_t r = 0; r < n; r++)
        std::memcpy(packed.data() + beg[r], idx.data() + off[r], (off[r + 1] - off[r]) * 4);
    c.slots = slots;
    c.max_cap = max_cap;
    *top = (uint32_t)pos;
    DFPR_HIP(hipMalloc(&c.beg, (size_t)n * 4));
    DFPR_HIP(hipMalloc(&c.cnt, (size_t)n * 4));
    DFPR_HIP(hipMalloc(&c.cap, (size_t)n * 4));
    DFPR_HIP(hipMalloc(&c.idx, slots * 4));
    DFPR_HIP(hipMemcpy(c.beg, beg.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    DFPR_HIP(hipMemcpy(c.cnt, cnt.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    DFPR_HIP(hipMemcpy(c.cap, cap.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    if (pos) DFPR_HIP(hipMemcpy(c.idx, packed.data(), pos * 4, hipMemcpyHostToDevice));
    return DFPR_OK;
}

static void free_csr(Csr &c)
{
    (void)hipFree(c.beg);
    (void)hipFree(c.cnt);
    (void)hipFree(c.cap);
    (void)hipFree(c.idx);
    c = Csr{};
}

// Internal numbering: decreasing in-degree counted over the input edges
// (repeats and self-loops included, which only affects ties), ties kept in
// the caller's order.  A counting sort by degree.
// Internal ids by decreasing in-degree (self-loop counted once, repeated
// input edges as given), stable in the caller's ids.  cls[] receives the id
// ranges of the in-degree classes in that order (see Ctl::cls).
static void renumber(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     std::vector<int32_t> &ext2int, std::vector<int32_t> &int2ext,
                     uint32_t cls[kBins + 2])
{
    std::vector<uint32_t> deg(n, 1);
    uint32_t dmax = 1;
    for (int64_t i = 0; i < m; i++) dmax = std::max(dmax, ++deg[dst[i]]);
    // class kBins - 1 - k starts at id cls[k]: count the rows above it
    uint64_t above[kBins + 1] = {};
    for (int32_t v = 0; v < n; v++) {
        const int b = bin_of(deg[v]);
        for (int k = 1; k < kBins; k++) above[k] += b > kBins - 1 - k ? 1 : 0;
        above[kBins] += deg[v] > 1 ? 1 : 0;
    }
    cls[0] = 0;
    for (int k = 1; k <= kBins; k++) cls[k] = (uint32_t)above[k];
    cls[kBins + 1] = (uint32_t)n;
    std::vector<uint64_t> start(dmax + 2, 0);
    for (int32_t v = 0; v < n; v++) start[dmax - deg[v] + 1]++;
    for (uint32_t d = 0; d <= dmax; d++) start[d + 1] += start[d];
    ext2int.assign(n, 0);
    int2ext.assign(n, 0);
    for (int32_t v = 0; v < n; v++) {
        const int32_t i = (int32_t)start[dmax - deg[v]]++;
        ext2int[v] = i;
        int2ext[i] = v;
    }
}

__global__ void k_map_ids(int32_t n, const int32_t *ext2int, const int32_t *in, int32_t *out,
                          int64_t len)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    const int32_t x = in[i];
    out[i] = (x >= 0 && x < n) ? ext2int[x] : -1;
}

// out[v] = Rint[ext2int[v]]: caller order from internal order
__global__ void k_to_caller(int32_t n, const int32_t *ext2int, const double *Rint, double *out)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) out[v] = Rint[ext2int[v]];
}

// Rint[i] = in[int2ext[i]]: internal order from caller order
__global__ void k_from_caller(int32_t n, const int32_t *int2ext, const double *in, double *Rint)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Rint[i] = in[int2ext[i]];
}

static inline unsigned grid_of(int64_t items)
{
    return (unsigned)std::max<int64_t>(1, (items + kBlock - 1) / kBlock);
}

// Four arrays of lengths l0..l3 mapped into consecutive ranges of `out`.
__global__ void k_map_ids4(int32_t n, const int32_t *ext2int, const int32_t *i0,
                           const int32_t *i1, const int32_t *i2, const int32_t *i3, int64_t l0,
                           int64_t l1, int64_t l2, int64_t l3, int32_t *out)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= l0 + l1 + l2 + l3) return;
    const int64_t k = i;
    const int32_t *src = i0;
    if (i >= l0) { i -= l0; src = i1;
        if (i >= l1) { i -= l1; src = i2;
            if (i >= l2) { i -= l2; src = i3; } } }
    const int32_t x = src[i];
    out[k] = (x >= 0 && x < n) ? ext2int[x] : -1;
}

int map_ids4(dfpr_graph *g, const int32_t *const in[4], const int64_t len[4], int32_t *out)
{
    const int64_t tot = len[0] + len[1] + len[2] + len[3];
    if (tot <= 0) return DFPR_OK;
    k_map_ids4<<<grid_of(tot), kBlock, 0, g->stream>>>(g->n, g->ext2int, in[0], in[1], in[2],
                                                       in[3], len[0], len[1], len[2], len[3], out);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

// Ids outside [0, n) become -1, which every later check rejects.  `in` may
// equal `out`.
int map_ids(dfpr_graph *g, const int32_t *in, int32_t *out, int64_t len)
{
    if (len <= 0) return DFPR_OK;
    k_map_ids<<<grid_of(len), kBlock, 0, g->stream>>>(g->n, g->ext2int, in, out, len);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

int ranks_to_caller(const dfpr_graph *g, const double *Rint, double *out, int out_dev)
{
    const int32_t n = g->n;
    k_to_caller<<<grid_of(n), kBlock, 0, g->stream>>>(n, g->ext2int, Rint, out_dev ? out : g->Rx);
    DFPR_HIP(hipGetLastError());
    if (!out_dev)
        DFPR_HIP(hipMemcpyAsync(out, g->Rx, (size_t)n * 8, hipMemcpyDeviceToHost, g->stream));
    return DFPR_OK;
}

int ranks_from_caller(const dfpr_graph *g, const double *in, int in_dev, double *Rint)
{
    const int32_t n = g->n;
    if (!in_dev) {
        DFPR_HIP(hipMemcpyAsync(g->Rx, in, (size_t)n * 8, hipMemcpyHostToDevice, g->stream));
        in = g->Rx;
    }
    k_from_caller<<<grid_of(n), kBlock, 0, g->stream>>>(n, g->int2ext, in, Rint);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

static int load_impl(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     dfpr_graph *g, uint32_t top[2])
{
    // out-rows: counting sort by source, self-loop included, then sort and
    // drop repeats inside each row
    std::vector<uint64_t> ooff(n + 1, 0);
    for (int64_t i = 0; i < m; i++) ooff[src[i] + 1]++;
    for (int32_t v = 0; v < n; v++) ooff[v + 1]++;
    for (int32_t v = 0; v < n; v++) ooff[v + 1] += ooff[v];
    std::vector<int32_t> oraw(ooff[n]);
    {
        std::vector<uint64_t> cur(ooff.begin(), ooff.end() - 1);
        for (int64_t i = 0; i < m; i++) oraw[cur[src[i]]++] = dst[i];
        for (int32_t v = 0; v < n; v++) oraw[cur[v]++] = v;
    }
    std::vector<uint64_t> oc(n + 1, 0);
    std::vector<int32_t> oidx;
    oidx.reserve(oraw.size());
    for (int32_t u = 0; u < n; u++) {
        auto b = oraw.begin() + ooff[u], e = oraw.begin() + ooff[u + 1];
        std::sort(b, e);
        auto ue = std::unique(b, e);
        oidx.insert(oidx.end(), b, ue);
        oc[u + 1] = oidx.size();
    }
    std::vector<int32_t>().swap(oraw);
    g->m = (int64_t)oidx.size();
    // in-rows: stable counting sort of the out-rows by destination; visiting
    // sources in increasing order leaves every in-row sorted
    std::vector<uint64_t> ic(n + 1, 0);
    for (int32_t v : oidx) ic[v + 1]++;
    for (int32_t v = 0; v < n; v++) ic[v + 1] += ic[v];
    std::vector<int32_t> iidx(oidx.size());
    {
        std::vector<uint64_t> cur(ic.begin(), ic.end() - 1);
        for (int32_t u = 0; u < n; u++)
            for (uint64_t k = oc[u]; k < oc[u + 1]; k++) iidx[cur[oidx[k]]++] = u;
    }
    int rc = upload_csr(g->csr[1], n, oc, oidx, &top[1]);
    if (rc) return rc;
    return upload_csr(g->csr[0], n, ic, iidx, &top[0]);
}

}  // namespace dfpr

using namespace dfpr;

extern "C" {

const char *dfpr_last_error(void) { return g_last_error.c_str(); }

void dfpr_params_default(dfpr_params *p)
{
    if (!p) return;
    p->alpha = 0.85;
    p->tol = 1e-10;
    p->frontier_tol = 1e-10 / 1e5;
    p->max_iters = 500;
    p->precision = DFPR_FP64;
    p->mode = DFPR_SYNC;
    p->loop = DFPR_LOOP_LAUNCHES;
}

void dfpr_free_graph(dfpr_graph *g)
{
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    free_csr(g->csr[0]);
    free_csr(g->csr[1]);
    for (int b = 0; b < 2; b++) {
        (void)hipFree(g->R[b]);
        (void)hipFree(g->C[b]);
        (void)hipFree(g->C32[b]);
    }
    (void)hipFree(g->stamp);
    (void)hipFree(g->xstamp);
    (void)hipFree(g->mstamp);
    (void)hipFree(g->mxstamp);
    (void)hipFree(g->bins);
    (void)hipFree(g->bfs_q);
    (void)hipFree(g->ctl);
    (void)hipFree(g->scratch_sum);
    (void)hipFree(g->Rx);
    (void)hipFree(g->ext2int);
    (void)hipFree(g->int2ext);
    if (g->ctl_host) (void)hipHostFree(g->ctl_host);
    if (g->ap.batch_host) (void)hipHostFree(g->ap.batch_host);
    (void)hipFree(g->it.dr_part);
    (void)hipFree(g->it.rmax_part);
    (void)hipFree(g->it.cnt_part);
    for (int o = 0; o < 2; o++) {
        for (int k = 0; k < 2; k++) (void)hipFree(g->ap.keys[o][k]);
        (void)hipFree(g->ap.tiny_list[o]);
        (void)hipFree(g->ap.small_list[o]);
        (void)hipFree(g->ap.big_list[o]);
        (void)hipFree(g->ap.ovf_list[o]);
        (void)hipFree(g->ap.ovf_need[o]);
    }
    (void)hipFree(g->ap.part);
    (void)hipFree(g->ap.slab);
    (void)hipFree(g->ap.batch_dev);
    for (hipEvent_t e : {g->ev0, g->ev1, g->ev_mid, g->ev_a0, g->ev_a1})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->evk)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->evc)
        if (e) (void)hipEventDestroy(e);
    if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
    delete g;
}

int dfpr_load_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    dfpr_graph **out)
{
    if (!out) return set_error(DFPR_E_ARG, "out is NULL");
    *out = nullptr;
    if (n <= 0 || m < 0 || (m > 0 && (!src || !dst)))
        return set_error(DFPR_E_ARG, "need n >= 1, m >= 0 and non-NULL edge arrays");
    int rc = check_ids_host(n, m, src, dst);
    if (rc) return rc;
    dfpr_graph *g = new dfpr_graph();
    g->n = n;
    uint32_t top[2] = {0, 0};
    renumber(n, m, src, dst, g->ext2int_h, g->int2ext_h, g->cls);
    {
        std::vector<int32_t> s2(m), d2(m);
        for (int64_t i = 0; i < m; i++) {
            s2[i] = g->ext2int_h[src[i]];
            d2[i] = g->ext2int_h[dst[i]];
        }
        rc = load_impl(n, m, s2.data(), d2.data(), g, top);
    }
    if (!rc) {
        auto al = [&](void **p, size_t bytes) -> int {
            hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 4));
            return e == hipSuccess ? 0 : hip_fail(e, "hipMalloc");
        };
        size_t nd = (size_t)n * 8;
        for (int b = 0; b < 2 && !rc; b++) {
            rc = al((void **)&g->R[b], nd);
            if (!rc) rc = al((void **)&g->C[b], nd);
        }
        if (!rc) rc = al((void **)&g->stamp, (size_t)n * 4);
        if (!rc) rc = al((void **)&g->xstamp, (size_t)n * 4);
        if (!rc) rc = al((void **)&g->bins, (size_t)kBins * n * 4);
        if (!rc) rc = al((void **)&g->ctl, sizeof(Ctl));
        if (!rc) rc = al((void **)&g->it.dr_part, kFoldSlots * 8);
        if (!rc) rc = al((void **)&g->it.rmax_part, kFoldSlots * 8);
        if (!rc) rc = al((void **)&g->C32[0], (size_t)n * 4);
        if (!rc) rc = al((void **)&g->C32[1], (size_t)n * 4);
        if (!rc) rc = al((void **)&g->it.cnt_part, (size_t)kFoldSlots * kCounters * 8);
        // the fold slots start cleared; every fold clears them again
        if (!rc && (hipMemset(g->it.dr_part, 0, kFoldSlots * 8) != hipSuccess ||
                    hipMemset(g->it.rmax_part, 0, kFoldSlots * 8) != hipSuccess ||
                    hipMemset(g->it.cnt_part, 0, (size_t)kFoldSlots * kCounters * 8) != hipSuccess))
            rc = set_error(DFPR_E_DEVICE, "hipMemset of the fold slots failed");
        if (!rc) rc = al((void **)&g->scratch_sum, 4096 * 8);
        if (!rc) rc = al((void **)&g->Rx, nd);
        if (!rc) rc = al((void **)&g->ext2int, (size_t)n * 4);
        if (!rc) rc = al((void **)&g->int2ext, (size_t)n * 4);
        if (!rc && hipMemcpy(g->ext2int, g->ext2int_h.data(), (size_t)n * 4,
                             hipMemcpyHostToDevice) != hipSuccess)
            rc = set_error(DFPR_E_DEVICE, "map upload failed");
        if (!rc && hipMemcpy(g->int2ext, g->int2ext_h.data(), (size_t)n * 4,
                             hipMemcpyHostToDevice) != hipSuccess)
            rc = set_error(DFPR_E_DEVICE, "map upload failed");
    }
    if (!rc) {
        // two mirrors: the chunk in flight in each slot of the iteration loop
        hipError_t e =
            hipHostMalloc((void **)&g->ctl_host, 2 * sizeof(Ctl), hipHostMallocCoherent);
        if (e != hipSuccess) rc = hip_fail(e, "hipHostMalloc");
    }
    if (!rc) {
        hipError_t e = hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&g->ev0);
        if (e == hipSuccess) e = hipEventCreate(&g->ev1);
        // phase marks, read after the call's stream synchronisation
        for (hipEvent_t *ev : {&g->ev_mid, &g->ev_a0, &g->ev_a1})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
        // per-launch timing only, read after a stream synchronisation: no
        // system-scope fence (with it, each record stalls the queue ~6 us)
        for (hipEvent_t &ev : g->evk)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
        // waited on before the host reads a chunk's mirror: keep the fence
        for (hipEvent_t &ev : g->evc)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e, "stream/event");
        g->stream = g->own_stream;
    }
    if (!rc) {
        (void)hipGetDevice(&g->device);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, g->device) == hipSuccess && prop.multiProcessorCount > 0)
        {
            g->grid = std::min(kMaxGrid, prop.multiProcessorCount * kGridPerCU);
            g->grid_wide = std::min(kMaxGrid, prop.multiProcessorCount * kWideGridPerCU);
            g->grid_wide_df = std::min(kMaxGrid, prop.multiProcessorCount * kWideDfGridPerCU);
        }
        int coop = 0;
        if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device) ==
            hipSuccess)
            g->coop = coop ? 1 : 0;
    }
    if (!rc) {
        Ctl c0;
        std::memset(&c0, 0, sizeof(c0));
        for (int o = 0; o < 2; o++) {
            c0.top[o] = top[o];
            c0.max_cap[o] = g->csr[o].max_cap;
        }
        for (int k = 0; k < kBins + 2; k++) c0.cls[k] = g->cls[k];
        hipError_t e = hipMemcpy(g->ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy");
        g->sparse_limit = (uint32_t)std::max<int64_t>(4096, n / 64);
    }
    if (!rc) rc = launch_fill_u32(g, g->stamp, (uint64_t)n, 0);
    if (!rc) rc = launch_fill_u32(g, g->xstamp, (uint64_t)n, 0);
    if (!rc) rc = dfpr_set_ranks(g, nullptr, 0);   // uniform 1/n
    if (!rc) {
        hipError_t e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    if (rc) {
        dfpr_free_graph(g);
        return rc;
    }
    *out = g;
    return DFPR_OK;
}

int dfpr_set_stream(dfpr_graph *g, void *hip_stream)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    DFPR_HIP(hipStreamSynchronize(g->stream));
    g->stream = hip_stream ? (hipStream_t)hip_stream : g->own_stream;
    return DFPR_OK;
}

int dfpr_graph_info(const dfpr_graph *g, int32_t *n, int64_t *m)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    return DFPR_OK;
}

int dfpr_export_csr(const dfpr_graph *g, int out_orientation, int64_t *offsets, int32_t *idx)
{
    if (!g || !offsets || !idx) return set_error(DFPR_E_ARG, "NULL argument");
    const Csr &c = g->csr[out_orientation ? 1 : 0];
    int32_t n = g->n;
    std::vector<uint32_t> beg(n), cnt(n);
    std::vector<int32_t> slots(c.slots);
    DFPR_HIP(hipStreamSynchronize(g->stream));
    DFPR_HIP(hipMemcpy(beg.data(), c.beg, (size_t)n * 4, hipMemcpyDeviceToHost));
    DFPR_HIP(hipMemcpy(cnt.data(), c.cnt, (size_t)n * 4, hipMemcpyDeviceToHost));
    DFPR_HIP(hipMemcpy(slots.data(), c.idx, c.slots * 4, hipMemcpyDeviceToHost));
    // rows and entries in the caller's numbering, entries ascending
    int64_t pos = 0;
    for (int32_t v = 0; v < n; v++) {
        const int32_t r = g->ext2int_h[v];
        offsets[v] = pos;
        if (pos + cnt[r] > g->m)
            return set_error(DFPR_E_DEVICE, "device CSR holds more entries than m");
        if ((uint64_t)beg[r] + cnt[r] > (uint64_t)c.slots)
            return set_error(DFPR_E_DEVICE, "device CSR row runs past its slots");
        for (uint32_t k = 0; k < cnt[r]; k++) idx[pos + k] = g->int2ext_h[slots[beg[r] + k]];
        std::sort(idx + pos, idx + pos + cnt[r]);
        pos += cnt[r];
    }
    offsets[n] = pos;
    if (pos != g->m) return set_error(DFPR_E_DEVICE, "device CSR entry count differs from m");
    return DFPR_OK;
}

int dfpr_get_ranks(const dfpr_graph *g, double *ranks, int on_device)
{
    if (!g || !ranks) return set_error(DFPR_E_ARG, "NULL argument");
    const int rc = ranks_to_caller(g, g->R[g->cur], ranks, on_device);
    if (rc) return rc;
    DFPR_HIP(hipStreamSynchronize(g->stream));
    return DFPR_OK;
}

}  // extern "C"
