// Rank engines: Static, Naive-dynamic and Dynamic Frontier PageRank.
//
// One iteration of every engine is one launch of k_iter, which
//   - pulls Eq. 1 for the rows in the class lists (the affected vertices of
//     Algorithm 1, or every vertex for Static / Naive-dynamic), a row being
//     reduced by a group of 4..64 lanes or a whole workgroup according to its
//     in-degree class;
//   - computes Delta r = |r - R[v]| and the block's L-inf maximum;
//   - (Dynamic Frontier) marks the out-neighbours of every row whose rank
//     moved by more than frontier_tol and appends newly marked vertices to
//     their class lists, for the next iteration;
//   - has its last workgroup reduce the per-workgroup partials and decide
//     convergence (Delta R <= tol) or the iteration cap.
// The host enqueues iterations in chunks and reads the stop flag between
// chunks; launches issued after the stop flag is set return at once.
//
// Ranks are double-buffered (synchronous form, Section 4.2).  Both buffers
// hold identical values for every vertex between calls; an iteration reads
// one and writes only its processed rows into the other.  Because the
// marks only grow within a call, a row that is not processed in iteration i
// was not processed earlier either, so the two buffers still agree there.
// The contribution C[v] = R[v] / |out(v)| is stored beside each rank so the
// pull gathers one value per in-edge.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace dfpr {

__device__ __constant__ int kRowsPerUnit[kBins] = {64, 32, 16, 8, 4, 1};

struct IterArgs {
    int32_t n;
    const uint32_t *in_beg, *in_cnt;
    const int32_t *in_idx;
    const uint32_t *out_beg, *out_cnt;
    const int32_t *out_idx;
    const double *Rc, *Cc;      // read
    double *Rn, *Cn;            // written
    uint8_t *flags;
    int32_t *bins;
    uint32_t stride;            // entries per class list (= n)
    Ctl *ctl;
    double *dr_part;
    unsigned long long *edges_part, *verts_part;
    double base;                // (1 - alpha) / n
    double alpha, tol, ftol;
    int32_t it, max_iters;
};

__device__ inline int lane_id() { return __lane_id(); }

// Set the mark of x; true if this call set it (0 -> 1).  Marks are bytes;
// the atomic works on the aligned 32-bit word that holds the byte.
__device__ inline bool mark_vertex(uint8_t *flags, int32_t x)
{
    if (flags[x]) return false;
    uint32_t *w = reinterpret_cast<uint32_t *>(flags + (x & ~3));
    uint32_t bit = 1u << ((x & 3) * 8);
    uint32_t old = atomicOr(w, bit);
    return (old & bit) == 0;
}

// Wave-aggregated append of the lanes with `take` set to the class lists.
__device__ inline void append_to_bins(bool take, int32_t x, int cls, Ctl *ctl, int32_t *bins,
                                      uint32_t stride)
{
    unsigned long long pend = __ballot(take);
    const int lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    while (pend) {
        int leader = __ffsll((long long)pend) - 1;
        int c = __shfl(cls, leader);
        unsigned long long mine = __ballot(take && cls == c);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctl->live[c], (uint32_t)__popcll(mine));
        base = __shfl(base, leader);
        if (take && cls == c)
            bins[(size_t)c * stride + base + __popcll(mine & below)] = x;
        pend &= ~mine;
    }
}

// Mark every out-neighbour of w; all lanes of the wave take part.
__device__ inline void expand_vertex_wave(const IterArgs &a, int32_t w)
{
    const uint32_t ob = a.out_beg[w], oc = a.out_cnt[w];
    const int lane = lane_id();
    for (uint32_t base = 0; base < oc; base += kWave) {
        uint32_t k = base + lane;
        int32_t x = k < oc ? a.out_idx[ob + k] : 0;
        bool nw = k < oc && mark_vertex(a.flags, x);
        int cls = nw ? bin_of(a.in_cnt[x]) : 0;
        append_to_bins(nw, x, cls, a.ctl, a.bins, a.stride);
    }
}

// Same, with the whole workgroup striding over one long out-row.
__device__ inline void expand_vertex_block(const IterArgs &a, int32_t w)
{
    const uint32_t ob = a.out_beg[w], oc = a.out_cnt[w];
    for (uint32_t base = 0; base < oc; base += kBlock) {
        uint32_t k = base + threadIdx.x;
        int32_t x = k < oc ? a.out_idx[ob + k] : 0;
        bool nw = k < oc && mark_vertex(a.flags, x);
        int cls = nw ? bin_of(a.in_cnt[x]) : 0;
        append_to_bins(nw, x, cls, a.ctl, a.bins, a.stride);
    }
}

struct Acc {
    double dr_max = 0.0;
    unsigned long long edges = 0, verts = 0;
};

// Finish one row: Eq. 1, Delta r, writes, and the expansion decision.
template <bool EXPAND>
__device__ inline void finish_row(const IterArgs &a, int32_t v, uint32_t cnt, double s, Acc &acc,
                                  int32_t *q, uint32_t *qn)
{
    double r = a.base + a.alpha * s;
    double dr = fabs(r - a.Rc[v]);
    a.Rn[v] = r;
    a.Cn[v] = r / (double)a.out_cnt[v];
    acc.dr_max = fmax(acc.dr_max, dr);
    acc.edges += cnt;
    acc.verts += 1;
    if (EXPAND && dr > a.ftol) q[atomicAdd(qn, 1u)] = v;
}

// Rows first .. first + kBlock/G - 1 of a class list, G lanes per row.
// Each lane sums its strided share of the in-row in order, then the group
// folds the partial sums with a fixed butterfly; the order is a function of
// the row alone, so results are reproducible.
template <int G, bool EXPAND>
__device__ inline void pull_group(const IterArgs &a, const int32_t *list, uint32_t count,
                                  uint32_t first, Acc &acc, int32_t *q, uint32_t *qn)
{
    const int sub = threadIdx.x & (G - 1);
    const uint32_t pos = first + threadIdx.x / G;
    double s = 0.0;
    int32_t v = 0;
    uint32_t cnt = 0;
    if (pos < count) {
        v = list[pos];
        const uint32_t beg = a.in_beg[v];
        cnt = a.in_cnt[v];
        const int32_t *idx = a.in_idx + beg;
        uint32_t k = sub;
        for (; k + 3 * G < cnt; k += 4 * G) {
            int32_t i0 = idx[k], i1 = idx[k + G], i2 = idx[k + 2 * G], i3 = idx[k + 3 * G];
            double c0 = a.Cc[i0], c1 = a.Cc[i1], c2 = a.Cc[i2], c3 = a.Cc[i3];
            s += c0;
            s += c1;
            s += c2;
            s += c3;
        }
        for (; k < cnt; k += G) s += a.Cc[idx[k]];
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    if (pos < count && sub == 0) finish_row<EXPAND>(a, v, cnt, s, acc, q, qn);
}

// One heavy row, the whole workgroup.
template <bool EXPAND>
__device__ inline void pull_block(const IterArgs &a, int32_t v, Acc &acc, double *red, int32_t *q,
                                  uint32_t *qn)
{
    const uint32_t beg = a.in_beg[v], cnt = a.in_cnt[v];
    const int32_t *idx = a.in_idx + beg;
    double s = 0.0;
    uint32_t k = threadIdx.x;
    for (; k + 3 * kBlock < cnt; k += 4 * kBlock) {
        int32_t i0 = idx[k], i1 = idx[k + kBlock], i2 = idx[k + 2 * kBlock],
                i3 = idx[k + 3 * kBlock];
        double c0 = a.Cc[i0], c1 = a.Cc[i1], c2 = a.Cc[i2], c3 = a.Cc[i3];
        s += c0;
        s += c1;
        s += c2;
        s += c3;
    }
    for (; k < cnt; k += kBlock) s += a.Cc[idx[k]];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = ((red[0] + red[1]) + red[2]) + red[3];
        finish_row<EXPAND>(a, v, cnt, t, acc, q, qn);
    }
    __syncthreads();
}

template <bool EXPAND>
__global__ __launch_bounds__(kBlock) void k_iter(IterArgs a)
{
    __shared__ uint32_t s_cnt[kBins];
    __shared__ uint32_t s_ustart[kBins + 1];   // unit prefix, classes 5,4,...,0
    __shared__ double s_red[kBlock / kWave];
    __shared__ int32_t s_q[kBlock];
    __shared__ uint32_t s_qn;
    __shared__ int s_last;
    __shared__ double s_fdr[kBlock];
    __shared__ unsigned long long s_fe[kBlock], s_fv[kBlock];

    Ctl *ctl = a.ctl;
    if (ctl->done) return;
    const int par = a.it & 1;
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        s_ustart[0] = 0;
        for (int k = 0; k < kBins; k++) {
            int b = kBins - 1 - k;
            uint32_t c = ctl->snap[par][b];
            s_cnt[b] = c;
            acc += (c + kRowsPerUnit[b] - 1) / kRowsPerUnit[b];
            s_ustart[k + 1] = acc;
        }
        s_qn = 0;
    }
    __syncthreads();
    const uint32_t total = s_ustart[kBins];
    // workgroups past the work take no part; with no work at all, workgroup
    // 0 alone records the (empty) iteration
    const uint32_t active = max(1u, min((uint32_t)gridDim.x, total));
    if (blockIdx.x >= active) return;

    Acc acc;
    for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
        int k = 0;
        while (u >= s_ustart[k + 1]) k++;
        const int b = kBins - 1 - k;
        const uint32_t first = (u - s_ustart[k]) * kRowsPerUnit[b];
        const int32_t *list = a.bins + (size_t)b * a.stride;
        switch (b) {
        case 0: pull_group<4, EXPAND>(a, list, s_cnt[0], first, acc, s_q, &s_qn); break;
        case 1: pull_group<8, EXPAND>(a, list, s_cnt[1], first, acc, s_q, &s_qn); break;
        case 2: pull_group<16, EXPAND>(a, list, s_cnt[2], first, acc, s_q, &s_qn); break;
        case 3: pull_group<32, EXPAND>(a, list, s_cnt[3], first, acc, s_q, &s_qn); break;
        case 4: pull_group<64, EXPAND>(a, list, s_cnt[4], first, acc, s_q, &s_qn); break;
        default: pull_block<EXPAND>(a, list[first], acc, s_red, s_q, &s_qn); break;
        }
        if (EXPAND) {
            __syncthreads();
            const uint32_t nq = s_qn;
            if (nq) {
                const int wave = threadIdx.x / kWave;
                for (uint32_t i = wave; i < nq; i += kBlock / kWave) {
                    int32_t w = s_q[i];
                    if (a.out_cnt[w] <= 4096) expand_vertex_wave(a, w);
                }
                for (uint32_t i = 0; i < nq; i++) {
                    int32_t w = s_q[i];
                    if (a.out_cnt[w] > 4096) expand_vertex_block(a, w);
                }
                __syncthreads();
                if (threadIdx.x == 0) s_qn = 0;
            }
            __syncthreads();
        }
    }

    // workgroup partials
    s_fdr[threadIdx.x] = acc.dr_max;
    s_fe[threadIdx.x] = acc.edges;
    s_fv[threadIdx.x] = acc.verts;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s_fdr[threadIdx.x] = fmax(s_fdr[threadIdx.x], s_fdr[threadIdx.x + st]);
            s_fe[threadIdx.x] += s_fe[threadIdx.x + st];
            s_fv[threadIdx.x] += s_fv[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.dr_part[blockIdx.x] = s_fdr[0];
        a.edges_part[blockIdx.x] = s_fe[0];
        a.verts_part[blockIdx.x] = s_fv[0];
        uint32_t t = __hip_atomic_fetch_add(&ctl->ticket, 1u, __ATOMIC_ACQ_REL,
                                            __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == active - 1);
    }
    __syncthreads();
    if (!s_last) return;

    // last workgroup: reduce all partials, decide, prepare the next snapshot
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double dr = 0.0;
    unsigned long long e = 0, vv = 0;
    for (uint32_t i = threadIdx.x; i < active; i += kBlock) {
        dr = fmax(dr, __hip_atomic_load(&a.dr_part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        e += __hip_atomic_load(&a.edges_part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        vv += __hip_atomic_load(&a.verts_part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_fdr[threadIdx.x] = dr;
    s_fe[threadIdx.x] = e;
    s_fv[threadIdx.x] = vv;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s_fdr[threadIdx.x] = fmax(s_fdr[threadIdx.x], s_fdr[threadIdx.x + st]);
            s_fe[threadIdx.x] += s_fe[threadIdx.x + st];
            s_fv[threadIdx.x] += s_fv[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dR = s_fdr[0];
        ctl->edges += s_fe[0];
        ctl->verts += s_fv[0];
        ctl->iterations = a.it + 1;
        ctl->final_linf = dR;
        const bool conv = dR <= a.tol;
        if (conv) ctl->converged = 1;
        for (int b = 0; b < kBins; b++)
            ctl->snap[par ^ 1][b] =
                __hip_atomic_load(&ctl->live[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ctl->ticket = 0;
        if (conv || a.it + 1 >= a.max_iters) ctl->done = 1;
    }
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

// Clear the per-call loop state (not the batch-applier fields).
__global__ void k_reset(Ctl *ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int b = 0; b < kBins; b++) {
            ctl->live[b] = 0;
            ctl->snap[0][b] = ctl->snap[1][b] = 0;
        }
        ctl->ticket = 0;
        ctl->done = 0;
        ctl->iterations = 0;
        ctl->converged = 0;
        ctl->final_linf = 0.0;
        ctl->edges = ctl->verts = 0;
        ctl->err = 0;
        ctl->affected0 = 0;
    }
}

// Freeze the lists built by the marking as iteration 0's snapshot.
__global__ void k_snap(Ctl *ctl, int32_t max_iters)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long tot = 0;
        for (int b = 0; b < kBins; b++) {
            ctl->snap[0][b] = ctl->live[b];
            tot += ctl->live[b];
        }
        ctl->affected0 = tot;
        ctl->ticket = 0;
        ctl->done = (ctl->err || max_iters <= 0) ? 1 : 0;
    }
}

__global__ void k_fill_u8(uint8_t *p, uint64_t len)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// R[b][v] = (src ? src[v] : 1/n) and C[b][v] = R[b][v] / |out(v)|, b = 0, 1.
__global__ void k_init_ranks(int32_t n, const double *src, double *R0, double *R1, double *C0,
                             double *C1, const uint32_t *out_cnt)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double r = src ? src[v] : 1.0 / (double)n;
        double c = r / (double)out_cnt[v];
        R0[v] = r;
        R1[v] = r;
        C0[v] = c;
        C1[v] = c;
    }
}

__global__ void k_copy2(int32_t n, const double *a, double *a2, const double *b, double *b2)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        a2[v] = a[v];
        b2[v] = b[v];
    }
}

// Every vertex into its class list (Static and Naive-dynamic).
__global__ void k_mark_all(int32_t n, const uint32_t *in_cnt, Ctl *ctl, int32_t *bins,
                           uint32_t stride)
{
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    bool take = v < n;
    int cls = take ? bin_of(in_cnt[v]) : 0;
    append_to_bins(take, v, cls, ctl, bins, stride);
}

// Flag (and abort the loop) if a batch id lies outside [0, n).
__global__ void k_validate(int32_t n, int64_t nd, const int32_t *ds, const int32_t *dd,
                           int64_t ni, const int32_t *is, const int32_t *id, Ctl *ctl)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nd + ni) return;
    int32_t s = i < nd ? ds[i] : is[i - nd];
    int32_t d = i < nd ? dd[i] : id[i - nd];
    if (s < 0 || s >= n || d < 0 || d >= n) {
        atomicOr(&ctl->err, 1u);
        ctl->done = 1;
    }
}

// Initial marking (Section 4.1.1, Algorithm 1): one wave per batch edge
// (u, v) marks G^t.out(u), and for a deletion also v, which was in
// G^{t-1}.out(u).  The union is (G^{t-1} U G^t).out(u).
__global__ __launch_bounds__(kBlock) void k_mark_initial(int32_t n, int64_t nd, const int32_t *ds,
                                                         const int32_t *dd, int64_t ni,
                                                         const int32_t *is, const uint32_t *out_beg,
                                                         const uint32_t *out_cnt,
                                                         const int32_t *out_idx,
                                                         const uint32_t *in_cnt, uint8_t *flags,
                                                         Ctl *ctl, int32_t *bins, uint32_t stride)
{
    if (ctl->err) return;
    const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    if (w >= nd + ni) return;
    const int lane = lane_id();
    const int32_t u = w < nd ? ds[w] : is[w - nd];
    const uint32_t ob = out_beg[u], oc = out_cnt[u];
    for (uint32_t base = 0; base < oc; base += kWave) {
        uint32_t k = base + lane;
        int32_t x = k < oc ? out_idx[ob + k] : 0;
        bool nw = k < oc && mark_vertex(flags, x);
        int cls = nw ? bin_of(in_cnt[x]) : 0;
        append_to_bins(nw, x, cls, ctl, bins, stride);
    }
    if (w < nd) {
        int32_t x = dd[w];
        bool nw = lane == 0 && mark_vertex(flags, x);
        int cls = nw ? bin_of(in_cnt[x]) : 0;
        append_to_bins(nw, x, cls, ctl, bins, stride);
    }
}

// End of a Dynamic Frontier call: copy the processed rows of the result
// buffer into the other buffer and clear their marks.
__global__ void k_finish_listed(const Ctl *ctl, const int32_t *bins, uint32_t stride,
                                const double *Rres, double *Roth, const double *Cres, double *Coth,
                                uint8_t *flags, int copy_ranks)
{
    for (int b = 0; b < kBins; b++) {
        const uint32_t cnt = ctl->live[b];
        const int32_t *list = bins + (size_t)b * stride;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
             i += gridDim.x * blockDim.x) {
            int32_t v = list[i];
            if (copy_ranks) {
                Roth[v] = Rres[v];
                Coth[v] = Cres[v];
            }
            flags[v] = 0;
        }
    }
}

static inline int blocks_for(int64_t items, int per_block = kBlock)
{
    int64_t b = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65535 * 16));
}

int launch_fill_u8(dfpr_graph *g, uint8_t *p, uint64_t len)
{
    k_fill_u8<<<std::min<int>(blocks_for(len), 4096), kBlock, 0, g->stream>>>(p, len);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

struct BusyGuard {
    dfpr_graph *g;
    bool ok;
    explicit BusyGuard(dfpr_graph *g_) : g(g_) { ok = __atomic_exchange_n(&g->busy, 1, __ATOMIC_ACQ_REL) == 0; }
    ~BusyGuard()
    {
        if (ok) __atomic_store_n(&g->busy, 0, __ATOMIC_RELEASE);
    }
};

static int check_params(const dfpr_params *p, dfpr_params &out)
{
    if (p) out = *p;
    else dfpr_params_default(&out);
    if (!(out.alpha >= 0.0 && out.alpha < 1.0) || !(out.tol >= 0.0) ||
        !(out.frontier_tol >= 0.0) || out.max_iters < 0 ||
        (out.precision != DFPR_FP64 && out.precision != DFPR_FP32_KAHAN))
        return set_error(DFPR_E_ARG, "invalid parameters");
    return DFPR_OK;
}

static IterArgs iter_args(dfpr_graph *g, const dfpr_params &p)
{
    IterArgs a{};
    a.n = g->n;
    a.in_beg = g->csr[0].beg;
    a.in_cnt = g->csr[0].cnt;
    a.in_idx = g->csr[0].idx;
    a.out_beg = g->csr[1].beg;
    a.out_cnt = g->csr[1].cnt;
    a.out_idx = g->csr[1].idx;
    a.flags = g->flags;
    a.bins = g->bins;
    a.stride = (uint32_t)g->n;
    a.ctl = g->ctl;
    a.dr_part = g->it.dr_part;
    a.edges_part = g->it.edges_part;
    a.verts_part = g->it.verts_part;
    a.base = (1.0 - p.alpha) / (double)g->n;
    a.alpha = p.alpha;
    a.tol = p.tol;
    a.ftol = p.frontier_tol;
    a.max_iters = p.max_iters;
    return a;
}

// Run iterations until the device sets the stop flag.  Iteration i reads
// buffer (base ^ (i & 1)); returns the buffer holding the result.
static int run_loop(dfpr_graph *g, const dfpr_params &p, bool expand, int *res_buf)
{
    IterArgs a = iter_args(g, p);
    const int base = g->cur;
    int it = 0, chunk = 4;
    *res_buf = base;
    while (it < p.max_iters) {
        const int k = std::min(chunk, p.max_iters - it);
        for (int j = 0; j < k; j++) {
            const int i = it + j;
            const int src = base ^ (i & 1);
            a.Rc = g->R[src];
            a.Cc = g->C[src];
            a.Rn = g->R[src ^ 1];
            a.Cn = g->C[src ^ 1];
            a.it = i;
            if (expand)
                k_iter<true><<<g->grid, kBlock, 0, g->stream>>>(a);
            else
                k_iter<false><<<g->grid, kBlock, 0, g->stream>>>(a);
        }
        DFPR_HIP(hipGetLastError());
        DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, g->stream));
        DFPR_HIP(hipStreamSynchronize(g->stream));
        if (g->ctl_host->done) break;
        it += k;
        chunk = std::min(chunk * 2, 32);
    }
    if (p.max_iters == 0) {
        DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, g->stream));
        DFPR_HIP(hipStreamSynchronize(g->stream));
    }
    *res_buf = base ^ (g->ctl_host->iterations & 1);
    return DFPR_OK;
}

static void fill_stats(dfpr_graph *g, dfpr_stats *st, bool df)
{
    if (!st) return;
    const Ctl &c = *g->ctl_host;
    st->iterations = c.iterations;
    st->converged = c.converged;
    st->refine_sweeps = 0;
    st->reserved = 0;
    st->final_linf = c.final_linf;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev0, g->ev1);
    st->ms_device = ms;
    unsigned long long fin = 0;
    for (int b = 0; b < kBins; b++) fin += c.live[b];
    st->affected_initial = df ? (int64_t)c.affected0 : g->n;
    st->affected_final = df ? (int64_t)fin : g->n;
    st->vertices_processed = (int64_t)c.verts;
    st->edges_processed = (int64_t)c.edges;
}

// Static (prev == NULL, uniform start) or Naive-dynamic (start from prev,
// which may be the resident ranks).
static int full_sweeps(dfpr_graph *g, const dfpr_params *pp, const double *prev, int prev_dev,
                       bool use_resident, double *ranks_out, int out_dev, dfpr_stats *st)
{
    dfpr_params p;
    int rc = check_params(pp, p);
    if (rc) return rc;
    BusyGuard guard(g);
    if (!guard.ok) return set_error(DFPR_E_BUSY, "graph in use");
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    DFPR_HIP(hipEventRecord(g->ev0, s));
    const int cur = g->cur;
    if (prev) {
        DFPR_HIP(hipMemcpyAsync(g->R[cur], prev, (size_t)n * 8,
                                prev_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[cur], g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    } else if (!use_resident) {
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, nullptr, g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    }
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    k_mark_all<<<blocks_for(n), kBlock, 0, s>>>(n, g->csr[0].cnt, g->ctl, g->bins, (uint32_t)n);
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters);
    DFPR_HIP(hipGetLastError());
    int res = cur;
    rc = run_loop(g, p, false, &res);
    if (rc) return rc;
    k_copy2<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[res], g->R[res ^ 1], g->C[res],
                                             g->C[res ^ 1]);
    g->cur = res;
    DFPR_HIP(hipEventRecord(g->ev1, s));
    if (ranks_out)
        DFPR_HIP(hipMemcpyAsync(ranks_out, g->R[res], (size_t)n * 8,
                                out_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    fill_stats(g, st, false);
    return DFPR_OK;
}

static int df_impl(dfpr_graph *g, const dfpr_params *pp, int64_t nd, const int32_t *ds,
                   const int32_t *dd, int64_t ni, const int32_t *is, const int32_t *id,
                   int on_device, const double *prev, double *ranks_out, dfpr_stats *st)
{
    dfpr_params p;
    int rc = check_params(pp, p);
    if (rc) return rc;
    if (nd < 0 || ni < 0 || (nd && (!ds || !dd)) || (ni && (!is || !id)))
        return set_error(DFPR_E_ARG, "bad batch arrays");
    if (!on_device) {
        rc = check_ids_host(g->n, nd, ds, dd);
        if (!rc) rc = check_ids_host(g->n, ni, is, id);
        if (rc) return rc;
    }
    BusyGuard guard(g);
    if (!guard.ok) return set_error(DFPR_E_BUSY, "graph in use");
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    DFPR_HIP(hipEventRecord(g->ev0, s));
    const int32_t *bds = ds, *bdd = dd, *bis = is, *bid = id;
    if (!on_device) {
        rc = stage_batch(g, nd, ds, dd, ni, is, id, &bds, &bdd, &bis, &bid);
        if (rc) return rc;
    }
    const int cur = g->cur;
    if (prev) {
        DFPR_HIP(hipMemcpyAsync(g->R[cur], prev, (size_t)n * 8,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[cur], g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    }
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (nd + ni > 0) {
        k_validate<<<blocks_for(nd + ni), kBlock, 0, s>>>(n, nd, bds, bdd, ni, bis, bid, g->ctl);
        k_mark_initial<<<blocks_for((nd + ni) * kWave), kBlock, 0, s>>>(
            n, nd, bds, bdd, ni, bis, g->csr[1].beg, g->csr[1].cnt, g->csr[1].idx, g->csr[0].cnt,
            g->flags, g->ctl, g->bins, (uint32_t)n);
    }
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters);
    DFPR_HIP(hipGetLastError());
    int res = cur;
    rc = run_loop(g, p, true, &res);
    if (rc) return rc;
    if (g->ctl_host->err) {
        // nothing was marked or iterated; clear marks made before the check
        k_finish_listed<<<256, kBlock, 0, s>>>(g->ctl, g->bins, (uint32_t)n, nullptr, nullptr,
                                               nullptr, nullptr, g->flags, 0);
        DFPR_HIP(hipStreamSynchronize(s));
        return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
    }
    k_finish_listed<<<std::min(blocks_for(n), 2048), kBlock, 0, s>>>(
        g->ctl, g->bins, (uint32_t)n, g->R[res], g->R[res ^ 1], g->C[res], g->C[res ^ 1],
        g->flags, 1);
    g->cur = res;
    DFPR_HIP(hipEventRecord(g->ev1, s));
    if (ranks_out)
        DFPR_HIP(hipMemcpyAsync(ranks_out, g->R[res], (size_t)n * 8,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    fill_stats(g, st, true);
    return DFPR_OK;
}

}  // namespace dfpr

using namespace dfpr;

extern "C" {

int dfpr_set_ranks(dfpr_graph *g, const double *ranks, int on_device)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    if (ranks)
        DFPR_HIP(hipMemcpyAsync(g->R[0], ranks, (size_t)n * 8,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, ranks ? g->R[0] : nullptr, g->R[0], g->R[1],
                                                  g->C[0], g->C[1], g->csr[1].cnt);
    DFPR_HIP(hipGetLastError());
    g->cur = 0;
    DFPR_HIP(hipStreamSynchronize(s));
    return DFPR_OK;
}

int dfpr_pagerank_static(dfpr_graph *g, const dfpr_params *p, double *ranks_out, dfpr_stats *st)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    return full_sweeps(g, p, nullptr, 0, false, ranks_out, 0, st);
}

int dfpr_pagerank_naive_dynamic(dfpr_graph *g, const dfpr_params *p, const double *prev,
                                double *ranks_out, dfpr_stats *st)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    return full_sweeps(g, p, prev, 0, true, ranks_out, 0, st);
}

int dfpr_pagerank_dynamic_frontier(dfpr_graph *g, const dfpr_params *p, int64_t n_del,
                                   const int32_t *del_src, const int32_t *del_dst, int64_t n_ins,
                                   const int32_t *ins_src, const int32_t *ins_dst,
                                   const double *prev, double *ranks_out, dfpr_stats *st)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    return df_impl(g, p, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 0, prev, ranks_out, st);
}

int dfpr_pagerank_dynamic_frontier_device(dfpr_graph *g, const dfpr_params *p, int64_t n_del,
                                          const int32_t *del_src, const int32_t *del_dst,
                                          int64_t n_ins, const int32_t *ins_src,
                                          const int32_t *ins_dst, const double *prev,
                                          double *ranks_out, dfpr_stats *st)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    return df_impl(g, p, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 1, prev, ranks_out, st);
}

int dfpr_mark_affected(dfpr_graph *g, int64_t n_del, const int32_t *del_src,
                       const int32_t *del_dst, int64_t n_ins, const int32_t *ins_src,
                       const int32_t *ins_dst, uint8_t *flags_out)
{
    if (!g || !flags_out) return set_error(DFPR_E_ARG, "NULL argument");
    if (n_del < 0 || n_ins < 0 || (n_del && (!del_src || !del_dst)) ||
        (n_ins && (!ins_src || !ins_dst)))
        return set_error(DFPR_E_ARG, "bad batch arrays");
    int rc = check_ids_host(g->n, n_del, del_src, del_dst);
    if (!rc) rc = check_ids_host(g->n, n_ins, ins_src, ins_dst);
    if (rc) return rc;
    BusyGuard guard(g);
    if (!guard.ok) return set_error(DFPR_E_BUSY, "graph in use");
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    const int32_t *bds, *bdd, *bis, *bid;
    rc = stage_batch(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, &bds, &bdd, &bis, &bid);
    if (rc) return rc;
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (n_del + n_ins > 0)
        k_mark_initial<<<blocks_for((n_del + n_ins) * kWave), kBlock, 0, s>>>(
            n, n_del, bds, bdd, n_ins, bis, g->csr[1].beg, g->csr[1].cnt, g->csr[1].idx,
            g->csr[0].cnt, g->flags, g->ctl, g->bins, (uint32_t)n);
    DFPR_HIP(hipGetLastError());
    DFPR_HIP(hipMemcpyAsync(flags_out, g->flags, (size_t)n, hipMemcpyDeviceToHost, s));
    k_finish_listed<<<std::min(blocks_for(n), 2048), kBlock, 0, s>>>(
        g->ctl, g->bins, (uint32_t)n, nullptr, nullptr, nullptr, nullptr, g->flags, 0);
    DFPR_HIP(hipStreamSynchronize(s));
    return DFPR_OK;
}

int dfpr_get_affected(const dfpr_graph *g, uint8_t *flags_out)
{
    if (!g || !flags_out) return set_error(DFPR_E_ARG, "NULL argument");
    DFPR_HIP(hipStreamSynchronize(g->stream));
    Ctl c;
    DFPR_HIP(hipMemcpy(&c, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    std::fill(flags_out, flags_out + g->n, 0);
    std::vector<int32_t> list;
    for (int b = 0; b < kBins; b++) {
        list.resize(c.live[b]);
        if (c.live[b])
            DFPR_HIP(hipMemcpy(list.data(), g->bins + (size_t)b * g->n, (size_t)c.live[b] * 4,
                               hipMemcpyDeviceToHost));
        for (int32_t v : list) flags_out[v] = 1;
    }
    return DFPR_OK;
}

}  // extern "C"
