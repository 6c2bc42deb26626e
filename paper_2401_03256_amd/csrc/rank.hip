// Rank engines: Static, Naive-dynamic and Dynamic Frontier PageRank.
//
// One iteration of every engine is one launch of k_iter, which
//   - pulls Eq. 1 for the rows of the iteration: every vertex (Static,
//     Naive-dynamic) or the affected vertices (Dynamic Frontier);
//   - computes Delta r = |r - R[v]| and the L-inf maximum;
//   - (Dynamic Frontier) marks the out-neighbours of every row whose rank
//     moved by more than frontier_tol;
// followed by a one-workgroup launch of k_final that folds the
// per-workgroup partials and decides convergence (Delta R <= tol) or the
// iteration cap.
// The host enqueues iterations in chunks and reads the stop flag between
// chunks; launches issued after the stop flag is set return at once.
//
// Work layout.  Rows are split by in-degree into classes; a class-b row is
// reduced by group_of(b) lanes of one wave (1, 2, 4, 8, 32 or 64 lanes) or,
// above 1024 in-edges, by a whole workgroup.  Each lane loads kUnroll
// indices and then kUnroll contributions per round, so that many loads are
// in flight per wave.  Each lane sums its strided share of a row in order
// and the group folds the partial sums with a fixed butterfly, so the sum
// of a row depends on nothing but the row and its class.
//
// Marks.  stamp[v] holds the iteration, offset by a per-call base, from
// which v is affected: v is processed in iteration i iff
// base <= stamp[v] <= base + i.  Marks made in iteration i carry base+i+1,
// so they take effect from the next iteration (synchronous form), and a
// plain store suffices to make them.  Marks never go away within a call
// (Algorithm 1 has no unmarking step), and a vertex whose out-neighbours
// are all marked gains nothing from marking them again, so each vertex
// scans its out-row at most once per call (xstamp[v] == base afterwards).
//
// Two ways to walk the affected rows.  While few vertices are marked, the
// marking appends new vertices to per-class lists (sparse mode).  Once the
// lists pass a size limit, iterations walk the whole class schedule built
// from all vertices (sorted by id inside each class) and skip rows whose
// stamp is out of range (dense mode); marks are then plain stores.
//
// Ranks are double-buffered (synchronous form, Section 4.2).  Both buffers
// hold identical values between calls; an iteration reads one and writes
// only its processed rows into the other.  Because marks only grow within a
// call, a row not processed in iteration i was not processed earlier in the
// call either, so the two buffers still agree there.  The contribution
// C[v] = R[v] / |out(v)| is stored beside each rank so the pull gathers one
// value per in-edge.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace dfpr {

#ifndef DFPR_UNROLL
#define DFPR_UNROLL 4
#endif
#ifndef DFPR_ITER_MIN_BLOCKS
#define DFPR_ITER_MIN_BLOCKS 1
#endif
constexpr int kUnroll = DFPR_UNROLL;   // loads in flight per lane and round
constexpr int kSchedChunk = 4096;   // vertices per workgroup in the schedule build

struct IterArgs {
    int32_t n;
    const uint32_t *in_beg, *in_cnt;
    const int32_t *in_idx;
    const uint32_t *out_beg, *out_cnt;
    const int32_t *out_idx;
    const double *Rc, *Cc;      // read
    double *Rn, *Cn;            // written
    const float *C32c;          // FP32 contributions read (precision form)
    float *C32n;                // FP32 contributions written
    uint32_t *stamp, *xstamp;
    int32_t *bins;              // class lists (sparse mode), n entries each
    const int32_t *sched;       // class schedule of all vertices
    const uint32_t *sched_off;  // kBins + 1 offsets
    Ctl *ctl;
    double *dr_part;
    double *rmax_part;          // per-workgroup largest new rank
    unsigned long long *cnt_part;   // kCounters per workgroup
    double base_rank;           // (1 - alpha) / n
    double alpha, tol, ftol;
    uint32_t sbase;             // stamp base of the call
    uint32_t sparse_limit;
    int32_t it, max_iters;
    int32_t n_stride;
};

__device__ inline int lane_id() { return __lane_id(); }

struct Acc {
    double dr_max = 0.0;
    double r_max = 0.0;
    unsigned long long c[kCounters] = {0, 0, 0, 0};   // rows, edges, xrows, xedges
};

// Sum of the contributions of in-edges idx[k] for k = first, first + step,
// ... < cnt, added in that order.  FP64, or (F32) FP32 contributions added
// with Kahan's compensated summation and returned as sum - compensation in
// FP64.
template <bool F32>
__device__ inline double gather_sum(const IterArgs &a, const int32_t *idx, uint32_t first,
                                    uint32_t step, uint32_t cnt)
{
    if (!F32) {
        double s = 0.0;
        for (uint32_t k0 = first; k0 < cnt; k0 += step * kUnroll) {
            int32_t i[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++) {
                const uint32_t k = k0 + j * step;
                i[j] = k < cnt ? idx[k] : -1;
            }
            double c[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++) c[j] = i[j] >= 0 ? a.Cc[i[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < kUnroll; j++)
                if (i[j] >= 0) s += c[j];
        }
        return s;
    } else {
        float ks = 0.0f, kc = 0.0f;
        for (uint32_t k0 = first; k0 < cnt; k0 += step * kUnroll) {
            int32_t i[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++) {
                const uint32_t k = k0 + j * step;
                i[j] = k < cnt ? idx[k] : -1;
            }
            float c[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++) c[j] = i[j] >= 0 ? a.C32c[i[j]] : 0.0f;
#pragma unroll
            for (int j = 0; j < kUnroll; j++) {
                if (i[j] >= 0) {
                    const float y = c[j] - kc;
                    const float t = ks + y;
                    kc = (t - ks) - y;
                    ks = t;
                }
            }
        }
        return (double)ks - (double)kc;
    }
}

// Wave-aggregated append of the lanes with `take` set to the class lists.
// Every lane of the wave calls it.
__device__ inline void append_to_bins(bool take, int32_t x, int cls, Ctl *ctl, int32_t *bins,
                                      uint32_t stride)
{
    unsigned long long pend = __ballot(take);
    const int lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    while (pend) {
        const int leader = __ffsll((long long)pend) - 1;
        const int c = __shfl(cls, leader);
        const unsigned long long mine = __ballot(take && cls == c);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctl->live[c], (uint32_t)__popcll(mine));
        base = __shfl(base, leader);
        if (take && cls == c) bins[(size_t)c * stride + base + __popcll(mine & below)] = x;
        pend &= ~mine;
    }
}

// Mark the out-neighbours of w with stamp `sv`.  The calling lanes take
// positions lane0, lane0 + step, ... (lane0 < step); every lane of every
// calling wave runs the same number of rounds.
template <bool SPARSE>
__device__ inline void mark_out_row(const IterArgs &a, int32_t w, uint32_t lane0, uint32_t step,
                                    uint32_t sv)
{
    const uint32_t ob = a.out_beg[w], oc = a.out_cnt[w];
    for (uint32_t k0 = 0; k0 < oc; k0 += step * kUnroll) {
        int32_t x[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            const uint32_t k = k0 + lane0 + j * step;
            x[j] = k < oc ? a.out_idx[ob + k] : -1;
        }
        uint32_t st[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; j++) st[j] = x[j] >= 0 ? a.stamp[x[j]] : 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            bool nw = false;
            if (st[j] < a.sbase) {
                if (SPARSE) nw = atomicMax(&a.stamp[x[j]], sv) < a.sbase;
                else a.stamp[x[j]] = sv;
            }
            if (SPARSE) {
                const int cls = nw ? bin_of(a.in_cnt[x[j]]) : 0;
                append_to_bins(nw, x[j], cls, a.ctl, a.bins, a.n_stride);
            }
        }
    }
}

// Finish one row: Eq. 1, Delta r, writes; returns whether it must expand.
template <bool DF, bool F32>
__device__ inline bool finish_row(const IterArgs &a, int32_t v, uint32_t cnt, double s, double rc,
                                  uint32_t oc, Acc &acc)
{
    const double r = a.base_rank + a.alpha * s;
    const double dr = fabs(r - rc);
    a.Rn[v] = r;
    if (F32) a.C32n[v] = (float)(r / (double)oc);
    else a.Cn[v] = r / (double)oc;
    acc.dr_max = fmax(acc.dr_max, dr);
    acc.r_max = fmax(acc.r_max, r);
    acc.c[0] += 1;
    acc.c[1] += cnt;
    if (DF && dr > a.ftol && a.xstamp[v] != a.sbase) {
        a.xstamp[v] = a.sbase;
        acc.c[2] += 1;
        acc.c[3] += oc;
        return true;
    }
    return false;
}

// One wave unit: 64/G rows of a class list, G lanes per row.
template <int G, bool DF, bool F32>
__device__ inline void wave_unit(const IterArgs &a, const int32_t *list, uint32_t count,
                                 uint32_t first, bool check, bool sparse, Acc &acc)
{
    const int lane = lane_id();
    const int sub = lane & (G - 1);
    const uint32_t pos = first + lane / G;
    bool active = false;
    int32_t v = 0;
    uint32_t beg = 0, cnt = 0, oc = 1;
    double rc = 0.0;
    if (pos < count) {
        v = list[pos];
        beg = a.in_beg[v];
        cnt = a.in_cnt[v];
        if (sub == 0) {
            rc = a.Rc[v];
            oc = a.out_cnt[v];
        }
        active = true;
        if (DF && check) {
            const uint32_t st = a.stamp[v];
            active = st >= a.sbase && st <= a.sbase + (uint32_t)a.it;
        }
    }
    double s = 0.0;
    if (active) {
        if (cnt == 1) {
            // the self-loop is the only in-edge
            if (sub == 0) s = F32 ? (double)a.C32c[v] : a.Cc[v];
        } else {
            s = gather_sum<F32>(a, a.in_idx + beg, sub, G, cnt);
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    bool expand = false;
    if (active && sub == 0) expand = finish_row<DF, F32>(a, v, cnt, s, rc, oc, acc);
    if (DF) {
        unsigned long long q = __ballot(expand);
        const uint32_t sv = a.sbase + (uint32_t)a.it + 1;
        while (q) {
            const int l = __ffsll((long long)q) - 1;
            const int32_t w = __shfl(v, l);
            if (sparse) mark_out_row<true>(a, w, lane, kWave, sv);
            else mark_out_row<false>(a, w, lane, kWave, sv);
            q &= q - 1;
        }
    }
}

// One row of more than 1024 in-edges, the whole workgroup.  All threads
// call it with the same v.
template <bool DF, bool F32>
__device__ inline void block_row(const IterArgs &a, int32_t v, bool check, bool sparse, Acc &acc,
                                 double *red, int *flag)
{
    if (DF && check) {
        const uint32_t st = a.stamp[v];
        if (!(st >= a.sbase && st <= a.sbase + (uint32_t)a.it)) return;   // uniform
    }
    const uint32_t beg = a.in_beg[v], cnt = a.in_cnt[v];
    double s = gather_sum<F32>(a, a.in_idx + beg, threadIdx.x, kBlock, cnt);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = ((red[0] + red[1]) + red[2]) + red[3];
        *flag = finish_row<DF, F32>(a, v, cnt, t, a.Rc[v], a.out_cnt[v], acc) ? 1 : 0;
    }
    __syncthreads();
    if (DF && *flag) {
        const uint32_t sv = a.sbase + (uint32_t)a.it + 1;
        if (sparse) mark_out_row<true>(a, v, threadIdx.x, kBlock, sv);
        else mark_out_row<false>(a, v, threadIdx.x, kBlock, sv);
    }
    __syncthreads();
}

// Fold a max and kCounters sums over the workgroup; thread 0 gets the
// result.  Waves fold with shuffles, then the four wave results are
// combined in a fixed order.
__device__ inline void block_fold(double &dr, double &rm, unsigned long long (&c)[kCounters],
                                  double *wdr, double *wrm, unsigned long long (*wc)[kCounters])
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        dr = fmax(dr, __shfl_xor(dr, off, kWave));
        rm = fmax(rm, __shfl_xor(rm, off, kWave));
#pragma unroll
        for (int j = 0; j < kCounters; j++) c[j] += __shfl_xor(c[j], off, kWave);
    }
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) {
        wdr[wave] = dr;
        wrm[wave] = rm;
#pragma unroll
        for (int j = 0; j < kCounters; j++) wc[wave][j] = c[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWavesPerBlock; w++) {
            dr = fmax(dr, wdr[w]);
            rm = fmax(rm, wrm[w]);
#pragma unroll
            for (int j = 0; j < kCounters; j++) c[j] += wc[w][j];
        }
    }
    __syncthreads();
}

// Work of one iteration: per class, the list and its length; wave units
// of classes 5..0 in that order; block units are the class-6 rows.
struct Plan {
    uint32_t cnt[kBins];
    const int32_t *list[kBins];
    uint32_t ustart[kBins];
    uint32_t nwu, nbu;
};

__device__ inline void make_plan(const IterArgs &a, const Ctl *ctl, bool sparse, int par, Plan &p)
{
    for (int b = 0; b < kBins; b++) {
        if (sparse) {
            p.cnt[b] = ctl->snap[par][b];
            p.list[b] = a.bins + (size_t)b * a.n_stride;
        } else {
            p.cnt[b] = a.sched_off[b + 1] - a.sched_off[b];
            p.list[b] = a.sched + a.sched_off[b];
        }
    }
    uint32_t acc = 0;
    for (int k = 0; k < kBins - 1; k++) {
        const int b = kBins - 2 - k;
        const uint32_t rows = kWave / group_of(b);
        p.ustart[k] = acc;
        acc += (p.cnt[b] + rows - 1) / rows;
    }
    p.nwu = acc;
    p.nbu = p.cnt[kBins - 1];
}

// Workgroups that have work in an iteration: 0 .. active-1.  With no work
// at all, workgroup 0 alone records the (empty) iteration.
__device__ inline uint32_t active_blocks(const Plan &p, uint32_t grid)
{
    const uint32_t wblocks = (p.nwu + kWavesPerBlock - 1) / kWavesPerBlock;
    return max(1u, max(min(grid, p.nbu), min(grid, wblocks)));
}

template <bool DF, bool F32>
__global__ __launch_bounds__(kBlock, DFPR_ITER_MIN_BLOCKS) void k_iter(IterArgs a)
{
    __shared__ Plan s_plan;
    __shared__ double s_red[kWavesPerBlock];
    __shared__ int s_flag;
    __shared__ double s_wdr[kWavesPerBlock], s_wrm[kWavesPerBlock];
    __shared__ unsigned long long s_wc[kWavesPerBlock][kCounters];

    const Ctl *ctl = a.ctl;
    if (ctl->done || (F32 && ctl->phase_end)) return;
    const int par = a.it & 1;
    const bool sparse = DF && !ctl->dense;
    const bool check = DF && !sparse;
    if (threadIdx.x == 0) make_plan(a, ctl, sparse, par, s_plan);
    __syncthreads();
    const uint32_t G = gridDim.x;
    if (blockIdx.x >= active_blocks(s_plan, G)) return;
    const uint32_t nbu = s_plan.nbu, nwu = s_plan.nwu;

    Acc acc;
    for (uint32_t u = blockIdx.x; u < nbu; u += G)
        block_row<DF, F32>(a, s_plan.list[kBins - 1][u], check, sparse, acc, s_red, &s_flag);

    const int wave = threadIdx.x / kWave;
    for (uint32_t u = blockIdx.x * kWavesPerBlock + wave; u < nwu; u += G * kWavesPerBlock) {
        int k = 0;
        while (k + 1 < kBins - 1 && u >= s_plan.ustart[k + 1]) k++;
        const int b = kBins - 2 - k;
        const uint32_t first = (u - s_plan.ustart[k]) * (kWave / group_of(b));
        const int32_t *list = s_plan.list[b];
        const uint32_t cnt = s_plan.cnt[b];
        switch (b) {
        case 0: wave_unit<1, DF, F32>(a, list, cnt, first, check, sparse, acc); break;
        case 1: wave_unit<2, DF, F32>(a, list, cnt, first, check, sparse, acc); break;
        case 2: wave_unit<4, DF, F32>(a, list, cnt, first, check, sparse, acc); break;
        case 3: wave_unit<8, DF, F32>(a, list, cnt, first, check, sparse, acc); break;
        case 4: wave_unit<32, DF, F32>(a, list, cnt, first, check, sparse, acc); break;
        default: wave_unit<64, DF, F32>(a, list, cnt, first, check, sparse, acc); break;
        }
    }

    double dr = acc.dr_max, rm = acc.r_max;
    unsigned long long c[kCounters];
#pragma unroll
    for (int j = 0; j < kCounters; j++) c[j] = acc.c[j];
    block_fold(dr, rm, c, s_wdr, s_wrm, s_wc);
    if (threadIdx.x == 0) {
        a.dr_part[blockIdx.x] = dr;
        a.rmax_part[blockIdx.x] = rm;
#pragma unroll
        for (int j = 0; j < kCounters; j++) a.cnt_part[blockIdx.x * kCounters + j] = c[j];
    }
}

// After each iteration (one workgroup): fold the partials of the
// iteration's active workgroups, decide convergence or the cap, and prepare
// the next iteration.  The launch boundary orders it after k_iter.
// In the FP32 phase of the precision form, reaching tol or the FP32
// resolution of the ranks ends the phase instead of the call.
__global__ __launch_bounds__(kBlock) void k_final(IterArgs a, uint32_t grid, int df, int f32)
{
    __shared__ Plan s_plan;
    __shared__ double s_wdr[kWavesPerBlock], s_wrm[kWavesPerBlock];
    __shared__ unsigned long long s_wc[kWavesPerBlock][kCounters];
    Ctl *ctl = a.ctl;
    if (ctl->done || (f32 && ctl->phase_end)) return;
    const int par = a.it & 1;
    const bool sparse = df && !ctl->dense;
    if (threadIdx.x == 0) make_plan(a, ctl, sparse, par, s_plan);
    __syncthreads();
    const uint32_t active = active_blocks(s_plan, grid);
    double dr = 0.0, rm = 0.0;
    unsigned long long c[kCounters] = {0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < active; i += kBlock) {
        dr = fmax(dr, a.dr_part[i]);
        rm = fmax(rm, a.rmax_part[i]);
#pragma unroll
        for (int j = 0; j < kCounters; j++) c[j] += a.cnt_part[i * kCounters + j];
    }
    block_fold(dr, rm, c, s_wdr, s_wrm, s_wc);
    if (threadIdx.x == 0) {
        ctl->verts += c[0];
        ctl->edges += c[1];
        ctl->xverts += c[2];
        ctl->xedges += c[3];
        ctl->iterations = a.it + 1;
        ctl->final_linf = dr;
        if (sparse) {
            unsigned long long before = 0, after = 0;
            for (int b = 0; b < kBins; b++) {
                const uint32_t l = ctl->live[b];
                before += ctl->snap[par][b];
                after += l;
                ctl->snap[par ^ 1][b] = l;
            }
            ctl->marked += after - before;
            if (after > a.sparse_limit) ctl->dense = 1;
        }
        if (f32) {
            // FP32 contributions carry a relative rounding error of 2^-24;
            // changes below about 2^-22 of the largest rank are noise
            const double floor32 = rm * 0x1p-22;
            const bool stalled = ctl->phase_iters >= 3 && dr >= 0.97 * ctl->prev_linf;
            ctl->phase_iters += 1;
            if (dr <= a.tol || dr <= floor32 || stalled) ctl->phase_end = 1;
            if (a.it + 1 >= a.max_iters) ctl->done = 1;
        } else {
            const bool conv = dr <= a.tol;
            if (conv) ctl->converged = 1;
            if (conv || a.it + 1 >= a.max_iters) ctl->done = 1;
        }
        ctl->prev_linf = dr;
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
        ctl->done = 0;
        ctl->dense = 0;
        ctl->phase_end = 0;
        ctl->phase_iters = 0;
        ctl->prev_linf = 0.0;
        ctl->renorm_scale = 1.0;
        ctl->iterations = 0;
        ctl->converged = 0;
        ctl->final_linf = 0.0;
        ctl->edges = ctl->verts = 0;
        ctl->xverts = ctl->xedges = ctl->marked = 0;
        ctl->affected0 = ctl->affected = 0;
        ctl->err = 0;
    }
}

// Freeze the lists built by the marking as iteration 0's snapshot and pick
// the walk of the first iteration.
__global__ void k_snap(Ctl *ctl, int32_t max_iters, uint32_t sparse_limit, int dense)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long tot = 0;
        for (int b = 0; b < kBins; b++) {
            ctl->snap[0][b] = ctl->live[b];
            tot += ctl->live[b];
        }
        ctl->dense = (dense || tot > sparse_limit) ? 1 : 0;
        ctl->done = (ctl->err || max_iters <= 0) ? 1 : 0;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t len, uint32_t value)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// R[b][v] = (src ? src[v] : 1/n) and C[b][v] = R[b][v] / |out(v)|, b = 0, 1.
__global__ void k_init_ranks(int32_t n, const double *src, double *R0, double *R1, double *C0,
                             double *C1, const uint32_t *out_cnt)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const double r = src ? src[v] : 1.0 / (double)n;
        const double c = r / (double)out_cnt[v];
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

// Class schedule of all vertices: a stable counting sort by class, in three
// passes (per-workgroup class counts, one scan, scatter).  Thread t of
// workgroup w owns the kSchedChunk/kBlock consecutive vertices starting at
// w * kSchedChunk + t * (kSchedChunk / kBlock).
__device__ inline void sched_thread_counts(int32_t n, const uint32_t *in_cnt, uint32_t v0,
                                           uint32_t (&cnt)[kBins])
{
#pragma unroll
    for (int b = 0; b < kBins; b++) cnt[b] = 0;
    for (int j = 0; j < kSchedChunk / kBlock; j++) {
        const uint32_t v = v0 + j;
        if (v < (uint32_t)n) cnt[bin_of(in_cnt[v])]++;
    }
}

__global__ __launch_bounds__(kBlock) void k_sched_count(int32_t n, const uint32_t *in_cnt,
                                                        uint32_t *tmp, uint32_t nblocks)
{
    __shared__ uint32_t s[kBins][kBlock];
    uint32_t cnt[kBins];
    sched_thread_counts(n, in_cnt, blockIdx.x * kSchedChunk + threadIdx.x * (kSchedChunk / kBlock),
                        cnt);
#pragma unroll
    for (int b = 0; b < kBins; b++) s[b][threadIdx.x] = cnt[b];
    __syncthreads();
    if (threadIdx.x < kBins) {
        uint32_t t = 0;
        for (int i = 0; i < kBlock; i++) t += s[threadIdx.x][i];
        tmp[threadIdx.x * nblocks + blockIdx.x] = t;
    }
}

// Exclusive scan of the class-major count table; off[b] = start of class b.
__global__ __launch_bounds__(kBlock) void k_sched_scan(uint32_t *tmp, uint32_t nblocks,
                                                       uint32_t *off)
{
    __shared__ uint32_t s[kBlock];
    const uint32_t len = nblocks * kBins;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < len; b0 += kBlock) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < len ? tmp[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            const uint32_t t = threadIdx.x >= (uint32_t)o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < len) {
            const uint32_t ex = carry + s[threadIdx.x] - v;
            tmp[i] = ex;
            if (i % nblocks == 0) off[i / nblocks] = ex;
        }
        const uint32_t tot = s[kBlock - 1];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) off[kBins] = carry;
}

__global__ __launch_bounds__(kBlock) void k_sched_scatter(int32_t n, const uint32_t *in_cnt,
                                                          const uint32_t *tmp, uint32_t nblocks,
                                                          int32_t *sched)
{
    __shared__ uint32_t s[kBins][kBlock];
    const uint32_t v0 = blockIdx.x * kSchedChunk + threadIdx.x * (kSchedChunk / kBlock);
    uint32_t cnt[kBins];
    sched_thread_counts(n, in_cnt, v0, cnt);
#pragma unroll
    for (int b = 0; b < kBins; b++) s[b][threadIdx.x] = cnt[b];
    __syncthreads();
    // inclusive scan per class over the threads of the workgroup
    for (int o = 1; o < kBlock; o <<= 1) {
        uint32_t t[kBins];
#pragma unroll
        for (int b = 0; b < kBins; b++)
            t[b] = threadIdx.x >= (uint32_t)o ? s[b][threadIdx.x - o] : 0;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < kBins; b++) s[b][threadIdx.x] += t[b];
        __syncthreads();
    }
    uint32_t pos[kBins];
#pragma unroll
    for (int b = 0; b < kBins; b++)
        pos[b] = tmp[b * nblocks + blockIdx.x] + s[b][threadIdx.x] - cnt[b];
    for (int j = 0; j < kSchedChunk / kBlock; j++) {
        const uint32_t v = v0 + j;
        if (v < (uint32_t)n) sched[pos[bin_of(in_cnt[v])]++] = (int32_t)v;
    }
}

// Flag (and abort the loop) if a batch id lies outside [0, n).
__global__ void k_validate(int32_t n, int64_t nd, const int32_t *ds, const int32_t *dd,
                           int64_t ni, const int32_t *is, const int32_t *id, Ctl *ctl)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nd + ni) return;
    const int32_t s = i < nd ? ds[i] : is[i - nd];
    const int32_t d = i < nd ? dd[i] : id[i - nd];
    if (s < 0 || s >= n || d < 0 || d >= n) {
        atomicOr(&ctl->err, 1u);
        ctl->done = 1;
    }
}

// Initial marking (Section 4.1.1, Algorithm 1): one wave per batch edge
// (u, v) marks G^t.out(u), and for a deletion also v, which was in
// G^{t-1}.out(u); the union is (G^{t-1} U G^t).out(u).  The marks carry
// stamp base, i.e. they are processed from iteration 0.  u's out-row is now
// fully marked, so u never needs to scan it again in this call.  With
// `append`, newly marked vertices also go to the class lists.
__global__ __launch_bounds__(kBlock) void k_mark_initial(IterArgs a, int64_t nd, const int32_t *ds,
                                                         const int32_t *dd, int64_t ni,
                                                         const int32_t *is, int append)
{
    __shared__ unsigned long long s_new;
    if (a.ctl->err) return;
    if (threadIdx.x == 0) s_new = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    unsigned long long mine = 0;
    for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave; w < nd + ni;
         w += waves) {
        const int32_t u = w < nd ? ds[w] : is[w - nd];
        const uint32_t ob = a.out_beg[u], oc = a.out_cnt[u];
        const uint32_t len = oc + (w < nd ? 1u : 0u);
        for (uint32_t kb = 0; kb < len; kb += kWave) {
            const uint32_t k = kb + lane;
            int32_t x = -1;
            if (k < oc) x = a.out_idx[ob + k];
            else if (k < len) x = dd[w];
            bool nw = false;
            if (x >= 0 && a.stamp[x] < a.sbase) nw = atomicMax(&a.stamp[x], a.sbase) < a.sbase;
            const unsigned long long m = __ballot(nw);
            if (lane == 0) mine += __popcll(m);
            if (append) {
                const int cls = nw ? bin_of(a.in_cnt[x]) : 0;
                append_to_bins(nw, x, cls, a.ctl, a.bins, a.n_stride);
            }
        }
        if (lane == 0) a.xstamp[u] = a.sbase;
    }
    if (lane == 0 && mine) atomicAdd(&s_new, mine);
    __syncthreads();
    if (threadIdx.x == 0 && s_new) atomicAdd(&a.ctl->affected0, s_new);
}

// End of a Dynamic Frontier call: copy the rows processed in this call from
// the result buffer into the other buffer and count the marked vertices.
__global__ __launch_bounds__(kBlock) void k_finish(int32_t n, const uint32_t *stamp, uint32_t lo,
                                                   uint32_t hi, const double *Rres, double *Roth,
                                                   const double *Cres, double *Coth, Ctl *ctl)
{
    __shared__ unsigned long long s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t st = stamp[v];
        if (st >= lo && st <= hi) {
            mine++;
            Roth[v] = Rres[v];
            Coth[v] = Cres[v];
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, kWave);
    if (lane_id() == 0 && mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(&ctl->affected, s_cnt);
}

// Precision form: FP32 copies of the FP64 contributions, both buffers.
__global__ void k_c32_init(int32_t n, const double *C, float *A, float *B)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float c = (float)C[v];
        A[v] = c;
        B[v] = c;
    }
}

// Sum of the ranks in FP64 with a fixed order: each workgroup folds a fixed
// range with a fixed tree, then one workgroup folds the partials in order.
constexpr int kSumBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_sum_part(int32_t n, const double *R, double *part)
{
    __shared__ double s[kBlock];
    const int64_t chunk = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min<int64_t>(lo + chunk, n);
    double acc = 0.0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += kBlock) acc += R[v];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kBlock) void k_sum_final(const double *part, int nb, Ctl *ctl)
{
    __shared__ double s[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl->renorm_scale = s[0] > 0.0 ? 1.0 / s[0] : 1.0;
}

// R <- R / sum(R) in both buffers and FP64 contributions rebuilt from it.
__global__ void k_renorm(int32_t n, double *Rres, double *Roth, double *C0, double *C1,
                         const uint32_t *out_cnt, const Ctl *ctl)
{
    const double scale = ctl->renorm_scale;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const double r = Rres[v] * scale;
        const double c = r / (double)out_cnt[v];
        Rres[v] = r;
        Roth[v] = r;
        C0[v] = c;
        C1[v] = c;
    }
}

static inline int blocks_for(int64_t items, int per_block = kBlock)
{
    const int64_t b = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65535 * 16));
}

int launch_fill_u32(dfpr_graph *g, uint32_t *p, uint64_t len, uint32_t value)
{
    k_fill_u32<<<std::min<int>(blocks_for((int64_t)len), 4096), kBlock, 0, g->stream>>>(p, len,
                                                                                       value);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

struct BusyGuard {
    dfpr_graph *g;
    bool ok;
    explicit BusyGuard(dfpr_graph *g_) : g(g_)
    {
        ok = __atomic_exchange_n(&g->busy, 1, __ATOMIC_ACQ_REL) == 0;
    }
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
        !(out.frontier_tol >= 0.0) || out.max_iters < 0 || out.max_iters > 100000 ||
        (out.precision != DFPR_FP64 && out.precision != DFPR_FP32_KAHAN))
        return set_error(DFPR_E_ARG, "invalid parameters");
    return DFPR_OK;
}

static IterArgs iter_args(dfpr_graph *g, const dfpr_params &p, uint32_t sbase)
{
    IterArgs a{};
    a.n = g->n;
    a.in_beg = g->csr[0].beg;
    a.in_cnt = g->csr[0].cnt;
    a.in_idx = g->csr[0].idx;
    a.out_beg = g->csr[1].beg;
    a.out_cnt = g->csr[1].cnt;
    a.out_idx = g->csr[1].idx;
    a.stamp = g->stamp;
    a.xstamp = g->xstamp;
    a.bins = g->bins;
    a.sched = g->sched;
    a.sched_off = g->sched_off;
    a.ctl = g->ctl;
    a.dr_part = g->it.dr_part;
    a.rmax_part = g->it.rmax_part;
    a.cnt_part = g->it.cnt_part;
    a.base_rank = (1.0 - p.alpha) / (double)g->n;
    a.alpha = p.alpha;
    a.tol = p.tol;
    a.ftol = p.frontier_tol;
    a.sbase = sbase;
    a.sparse_limit = g->sparse_limit;
    a.max_iters = p.max_iters;
    a.n_stride = g->n;
    return a;
}

// Rebuild the class schedule if in-degrees changed since the last build.
static int ensure_schedule(dfpr_graph *g)
{
    if (!g->sched_dirty) return DFPR_OK;
    const uint32_t nb = (uint32_t)((g->n + kSchedChunk - 1) / kSchedChunk);
    hipStream_t s = g->stream;
    k_sched_count<<<nb, kBlock, 0, s>>>(g->n, g->csr[0].cnt, g->sched_tmp, nb);
    k_sched_scan<<<1, kBlock, 0, s>>>(g->sched_tmp, nb, g->sched_off);
    k_sched_scatter<<<nb, kBlock, 0, s>>>(g->n, g->csr[0].cnt, g->sched_tmp, nb, g->sched);
    DFPR_HIP(hipGetLastError());
    g->sched_dirty = 0;
    return DFPR_OK;
}

// Take a stamp base for a new call; stamps of earlier calls are all below it.
static int take_base(dfpr_graph *g, int32_t max_iters, uint32_t *base)
{
    const uint64_t span = (uint64_t)max_iters + 2;
    if ((uint64_t)g->next_base + span >= 0xF0000000ull) {
        int rc = launch_fill_u32(g, g->stamp, (uint64_t)g->n, 0);
        if (!rc) rc = launch_fill_u32(g, g->xstamp, (uint64_t)g->n, 0);
        if (rc) return rc;
        g->next_base = 1;
    }
    *base = g->next_base;
    g->next_base += (uint32_t)span;
    return DFPR_OK;
}

// Run iterations it0, it0+1, ... until the device sets the stop flag (or,
// in the FP32 phase, the phase-end flag).  The phase starts on buffer
// `base`; iteration i reads buffer base ^ ((i - it0) & 1).  *res_buf
// receives the buffer holding the result.  Iterations are enqueued in
// chunks; between chunks the host reads the control block once and sizes
// the next chunk from the observed geometric decay of Delta R, so few
// launches run after convergence.
static int run_loop(dfpr_graph *g, const dfpr_params &p, bool df, bool f32, uint32_t sbase,
                    int it0, int base, int *res_buf)
{
    IterArgs a = iter_args(g, p, sbase);
    int it = it0, chunk = 4;
    double prev_dr = -1.0;
    int prev_it = it0;
    *res_buf = base;
    while (it < p.max_iters) {
        const int k = std::min(chunk, p.max_iters - it);
        if (g->prof.enabled) DFPR_HIP(hipEventRecord(g->evk0, g->stream));
        for (int j = 0; j < k; j++) {
            const int i = it + j;
            const int src = base ^ ((i - it0) & 1);
            a.Rc = g->R[src];
            a.Cc = g->C[src];
            a.Rn = g->R[src ^ 1];
            a.Cn = g->C[src ^ 1];
            a.C32c = g->C32[src];
            a.C32n = g->C32[src ^ 1];
            a.it = i;
            if (!df) k_iter<false, false><<<g->grid, kBlock, 0, g->stream>>>(a);
            else if (f32) k_iter<true, true><<<g->grid, kBlock, 0, g->stream>>>(a);
            else k_iter<true, false><<<g->grid, kBlock, 0, g->stream>>>(a);
            k_final<<<1, kBlock, 0, g->stream>>>(a, (uint32_t)g->grid, df ? 1 : 0, f32 ? 1 : 0);
        }
        DFPR_HIP(hipGetLastError());
        if (g->prof.enabled) DFPR_HIP(hipEventRecord(g->evk1, g->stream));
        DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, g->stream));
        DFPR_HIP(hipStreamSynchronize(g->stream));
        if (g->prof.enabled) {
            float ms = 0.f;
            DFPR_HIP(hipEventElapsedTime(&ms, g->evk0, g->evk1));
            g->prof.ms += ms;
            g->prof.launches += k;
        }
        if (g->ctl_host->done || (f32 && g->ctl_host->phase_end)) break;
        it += k;
        const double dr = g->ctl_host->final_linf;
        const int its = g->ctl_host->iterations;
        int next = std::min(chunk * 2, 32);
        if (!f32 && prev_dr > 0.0 && dr > 0.0 && dr < prev_dr && its > prev_it && p.tol > 0.0) {
            const double rate = std::pow(dr / prev_dr, 1.0 / (its - prev_it));
            const double need = std::ceil(std::log(p.tol / dr) / std::log(rate));
            if (std::isfinite(need)) next = (int)std::min(64.0, std::max(1.0, need));
        }
        prev_dr = dr;
        prev_it = its;
        chunk = next;
    }
    if (p.max_iters <= it0) {
        DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, g->stream));
        DFPR_HIP(hipStreamSynchronize(g->stream));
    }
    const Ctl &c = *g->ctl_host;
    *res_buf = base ^ ((c.iterations - it0) & 1);
    if (g->prof.enabled) {
        const int64_t dv = (int64_t)c.verts - g->prof_base[0];
        const int64_t de = (int64_t)c.edges - g->prof_base[1];
        const int64_t dxv = (int64_t)c.xverts - g->prof_base[2];
        const int64_t dxe = (int64_t)c.xedges - g->prof_base[3];
        g->prof.rows += dv;
        g->prof.edges += de;
        g->prof.exp_rows += dxv;
        g->prof.exp_edges += dxe;
        // per processed row: schedule entry 4 B, row start and length 8 B,
        // R[v] 8 B, |out(v)| 4 B, R'[v] and C'[v] written 16 B (12 B with an
        // FP32 contribution) (+ its mark 4 B and expansion stamp 4 B in
        // Dynamic Frontier); per in-edge: index 4 B and the gathered
        // contribution (8 B, or 4 B in FP32); per expanding row: out-row
        // start and length 8 B; per scanned out-edge: index 4 B and the
        // target's mark 4 B
        const double row_bytes = (df ? 48.0 : 40.0) - (f32 ? 4.0 : 0.0);
        const double edge_bytes = f32 ? 8.0 : 12.0;
        g->prof.bytes += row_bytes * dv + edge_bytes * de + 8.0 * dxv + 8.0 * dxe;
        g->prof_base[0] = (int64_t)c.verts;
        g->prof_base[1] = (int64_t)c.edges;
        g->prof_base[2] = (int64_t)c.xverts;
        g->prof_base[3] = (int64_t)c.xedges;
    }
    return DFPR_OK;
}

static void fill_stats(dfpr_graph *g, dfpr_stats *st, bool df)
{
    if (!st) return;
    const Ctl &c = *g->ctl_host;
    st->iterations = c.iterations;
    st->converged = c.converged;
    st->refine_sweeps = g->refine_sweeps;
    st->reserved = 0;
    st->final_linf = c.final_linf;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev0, g->ev1);
    st->ms_device = ms;
    st->affected_initial = df ? (int64_t)c.affected0 : g->n;
    st->affected_final = df ? (int64_t)c.affected : g->n;
    st->vertices_processed = (int64_t)c.verts;
    st->edges_processed = (int64_t)c.edges;
}

// Static (prev == NULL and !use_resident: uniform start) or Naive-dynamic
// (start from prev, or from the resident ranks).
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
    rc = ensure_schedule(g);
    if (rc) return rc;
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters, g->sparse_limit, 1);
    DFPR_HIP(hipGetLastError());
    int res = cur;
    g->refine_sweeps = 0;
    std::memset(g->prof_base, 0, sizeof(g->prof_base));
    rc = run_loop(g, p, false, false, 0, 0, cur, &res);
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
    rc = ensure_schedule(g);
    uint32_t sbase = 0;
    if (!rc) rc = take_base(g, p.max_iters, &sbase);
    if (rc) return rc;
    // a batch whose sources reach many vertices starts on the full schedule
    const double reach = (double)(nd + ni) * ((double)g->m / (double)n);
    const int dense = reach > (double)g->sparse_limit ? 1 : 0;
    IterArgs a = iter_args(g, p, sbase);
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (nd + ni > 0) {
        k_validate<<<blocks_for(nd + ni), kBlock, 0, s>>>(n, nd, bds, bdd, ni, bis, bid, g->ctl);
        k_mark_initial<<<std::min(blocks_for((nd + ni) * kWave), 2048), kBlock, 0, s>>>(
            a, nd, bds, bdd, ni, bis, dense ? 0 : 1);
    }
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters, g->sparse_limit, dense);
    DFPR_HIP(hipGetLastError());
    int res = cur;
    g->refine_sweeps = 0;
    std::memset(g->prof_base, 0, sizeof(g->prof_base));
    if (p.precision == DFPR_FP32_KAHAN) {
        // FP32 phase on FP32 copies of the contributions
        k_c32_init<<<blocks_for(n), kBlock, 0, s>>>(n, g->C[cur], g->C32[0], g->C32[1]);
        rc = run_loop(g, p, true, true, sbase, 0, cur, &res);
        if (rc) return rc;
        if (g->ctl_host->err)
            return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
        if (g->ctl_host->done) {
            // the cap ended the call inside the FP32 phase: rebuild the FP64
            // contributions (and the second buffer) from the ranks
            k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[res], g->R[0], g->R[1],
                                                          g->C[0], g->C[1], g->csr[1].cnt);
        } else {
            // renormalise to sum 1 and continue in FP64 over the same marks
            const int it0 = g->ctl_host->iterations;
            k_sum_part<<<kSumBlocks, kBlock, 0, s>>>(n, g->R[res], g->scratch_sum);
            k_sum_final<<<1, kBlock, 0, s>>>(g->scratch_sum, kSumBlocks, g->ctl);
            k_renorm<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[res], g->R[res ^ 1], g->C[0],
                                                      g->C[1], g->csr[1].cnt, g->ctl);
            DFPR_HIP(hipGetLastError());
            const int base2 = res;
            rc = run_loop(g, p, true, false, sbase, it0, base2, &res);
            if (rc) return rc;
            g->refine_sweeps = g->ctl_host->iterations - it0;
        }
    } else {
        rc = run_loop(g, p, true, false, sbase, 0, cur, &res);
        if (rc) return rc;
    }
    const int32_t iters = g->ctl_host->iterations;
    if (g->ctl_host->err) return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
    k_finish<<<std::min(blocks_for(n), 2048), kBlock, 0, s>>>(
        n, g->stamp, sbase, sbase + (uint32_t)iters, g->R[res], g->R[res ^ 1], g->C[res],
        g->C[res ^ 1], g->ctl);
    g->cur = res;
    g->last_base = sbase;
    g->last_iters = iters;
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
    dfpr_params p;
    dfpr_params_default(&p);
    uint32_t sbase = 0;
    if (!rc) rc = take_base(g, 0, &sbase);
    if (rc) return rc;
    IterArgs a = iter_args(g, p, sbase);
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (n_del + n_ins > 0)
        k_mark_initial<<<std::min(blocks_for((n_del + n_ins) * kWave), 2048), kBlock, 0, s>>>(
            a, n_del, bds, bdd, n_ins, bis, 0);
    DFPR_HIP(hipGetLastError());
    std::vector<uint32_t> st(n);
    DFPR_HIP(hipMemcpyAsync(st.data(), g->stamp, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    for (int32_t v = 0; v < n; v++) flags_out[v] = st[v] == sbase ? 1 : 0;
    return DFPR_OK;
}

int dfpr_get_affected(const dfpr_graph *g, uint8_t *flags_out)
{
    if (!g || !flags_out) return set_error(DFPR_E_ARG, "NULL argument");
    const int32_t n = g->n;
    std::vector<uint32_t> st(n);
    DFPR_HIP(hipStreamSynchronize(g->stream));
    DFPR_HIP(hipMemcpy(st.data(), g->stamp, (size_t)n * 4, hipMemcpyDeviceToHost));
    const uint32_t lo = g->last_base, hi = g->last_base + (uint32_t)std::max(g->last_iters, 0);
    for (int32_t v = 0; v < n; v++)
        flags_out[v] = (g->last_iters >= 0 && st[v] >= lo && st[v] <= hi) ? 1 : 0;
    return DFPR_OK;
}

int dfpr_profile_reset(dfpr_graph *g, int enable)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    g->prof = Profile{};
    g->prof.enabled = enable ? 1 : 0;
    return DFPR_OK;
}

int dfpr_profile_read(const dfpr_graph *g, dfpr_profile *out)
{
    if (!g || !out) return set_error(DFPR_E_ARG, "NULL argument");
    out->launches = g->prof.launches;
    out->ms = g->prof.ms;
    out->bytes = g->prof.bytes;
    out->rows = g->prof.rows;
    out->edges = g->prof.edges;
    out->expanded_rows = g->prof.exp_rows;
    out->expanded_edges = g->prof.exp_edges;
    out->marked = g->prof.marked;
    return DFPR_OK;
}

}  // extern "C"
