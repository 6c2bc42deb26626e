// Device code of one PageRank iteration, shared by the single-graph
// engines (rank.hip) and the multi-graph serving loop (serve.hip).  The
// layout and the marking rules are described at the top of rank.hip.
#pragma once

#include "common.h"

namespace dfpr {

// Index loads in flight per lane and round of a gather (each lane still
// adds its entries in index order, so the value does not change the sums).
// Measured on R-MAT scale 22: 8 beats 4, 6, 10, 12 and 16.
#ifndef DFPR_UNROLL
#define DFPR_UNROLL 8
#endif
// Minimum waves per SIMD the iteration kernels are compiled for (the second
// launch bound).  The kernels now fit 6-7 waves without spills; asking for
// eight is slower on R-MAT scale 22.
#ifndef DFPR_ITER_WAVES_PER_SIMD
#define DFPR_ITER_WAVES_PER_SIMD 5
#endif
// Index loads are streamed once per iteration; marking them non-temporal
// leaves more of L2 to the gathered contributions (4% on R-MAT scale 22;
// the same marking on the gathers themselves halves the speed).
#ifndef DFPR_NT_IDX
#define DFPR_NT_IDX 1
#endif
constexpr int kUnroll = DFPR_UNROLL;   // loads in flight per lane and round

// Streamed index loads: marked non-temporal so that they do not displace
// gathered contributions from L2.
__device__ __forceinline__ int32_t load_idx(const int32_t *p)
{
#if DFPR_NT_IDX
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Contributions of the first kHubRows vertices (the highest in-degrees, and
// with them the most out-edges) are copied into LDS by each workgroup of a
// sweep that walks the full schedule, and gathers from those sources read
// LDS instead of going through the vector L1 and L2.  On R-MAT scale 22 the
// first 2048 sources take 17% of the gathers; 16 KB per workgroup keeps
// seven workgroups per CU, and a static sweep runs 4.5% faster (4096
// entries halve the workgroups per CU and are slower).  0 switches it off.
#ifndef DFPR_HUB
#define DFPR_HUB 2048
#endif
constexpr uint32_t kHubRows = DFPR_HUB;

// The LDS copy a workgroup gathers from: n entries (0: none).
struct Hub {
    const double *d;    // FP64 contributions
    const float *f;     // FP32 contributions (precision form)
    uint32_t n;
};

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
    Ctl *ctl;
    Ctl *mirror;                // host-visible copy of the control block, or NULL
    double *dr_part;            // kFoldSlots slots of the L-inf of Delta r
    double *rmax_part;          //   ... of the largest new rank
    unsigned long long *cnt_part;   // kCounters per slot
    double base_rank;           // (1 - alpha) / n
    double alpha, tol, ftol;
    uint32_t sbase;             // stamp base of the call
    uint32_t sparse_limit;
    int32_t it, max_iters;
    int32_t n_stride;
    uint32_t hub;               // contributions to copy into LDS (0: none)
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// In-degree class of internal id v (its id range, Ctl::cls; the self-loop
// rows are in class 0).
__device__ __forceinline__ int class_of_id(const IterArgs &a, int32_t v)
{
    int c = kBins - 1;
#pragma unroll
    for (int k = 1; k < kBins; k++) c -= (uint32_t)v >= a.ctl->cls[k] ? 1 : 0;
    return c;
}

struct Acc {
    double dr_max = 0.0;
    double r_max = 0.0;
    // rows, edges, xrows, xedges of this lane: each below the graph's edge
    // slots (under 2^32), so 32 bits per lane; widened for the fold
    uint32_t c[kCounters] = {0, 0, 0, 0};
    double ftol = 0.0;          // frontier tolerance in effect
    bool plain = false;         // expansions mark with plain stores (Ctl::plain_marks)
};

// Sum of the contributions of in-edges idx[k] for k = first, first + step,
// ... < cnt, added in that order.  FP64, or (F32) FP32 contributions added
// with Kahan's compensated summation and returned as sum - compensation in
// FP64.
template <bool F32>
__device__ __forceinline__ double gather_sum(const IterArgs &a, const Hub &hub, const int32_t *idx,
                                    uint32_t first, uint32_t step, uint32_t cnt)
{
    if (!F32) {
        double s = 0.0;
        for (uint32_t k0 = first; k0 < cnt; k0 += step * kUnroll) {
            int32_t i[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++) {
                const uint32_t k = k0 + j * step;
                i[j] = k < cnt ? load_idx(idx + k) : -1;
            }
            double c[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++)
                c[j] = i[j] < 0 ? 0.0 : (uint32_t)i[j] < hub.n ? hub.d[i[j]] : a.Cc[i[j]];
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
                i[j] = k < cnt ? load_idx(idx + k) : -1;
            }
            float c[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; j++)
                c[j] = i[j] < 0 ? 0.0f : (uint32_t)i[j] < hub.n ? hub.f[i[j]] : a.C32c[i[j]];
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
__device__ __forceinline__ void append_to_bins(bool take, int32_t x, int cls, Ctl *ctl, int32_t *bins,
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
__device__ __forceinline__ void mark_out_row(const IterArgs &a, int32_t w, uint32_t lane0, uint32_t step,
                                    uint32_t sv)
{
    const uint32_t ob = a.out_beg[w], oc = a.out_cnt[w];
    for (uint32_t k0 = 0; k0 < oc; k0 += step * kUnroll) {
        int32_t x[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            const uint32_t k = k0 + lane0 + j * step;
            x[j] = k < oc ? load_idx(a.out_idx + ob + k) : -1;
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
                const int cls = nw ? class_of_id(a, x[j]) : 0;
                append_to_bins(nw, x[j], cls, a.ctl, a.bins, a.n_stride);
            }
        }
    }
}

// On the class lists, a row with more out-edges than this marks them with
// plain stores, like the full schedule does, and moves the call to the full
// schedule from the next iteration on: its out-row alone would fill a good
// part of the lists, and one workgroup appending them entry by entry (an
// atomic per out-edge) stalls the whole iteration.
__device__ __forceinline__ bool heavy_in_sparse(const IterArgs &a, uint32_t oc)
{
    return oc > a.sparse_limit / 8;
}

// Expansion of the rows of a wave whose lanes have `deg` > 0 out-edges
// starting at `ob` (`incl` = inclusive prefix sum of `deg` over the wave,
// `total` its last value): every lane takes one out-edge per round, so
// rows with few out-edges share rounds and list appends.  Every lane of
// the wave calls it with the same `total`.
template <bool SPARSE>
__device__ __forceinline__ void expand_rows(const IterArgs &a, uint32_t incl, uint32_t deg, uint32_t ob,
                                   uint32_t total, uint32_t sv)
{
    const int lane = lane_id();
    for (uint32_t t0 = 0; t0 < total; t0 += kWave) {
        const uint32_t t = t0 + lane;
        const uint32_t tt = min(t, total - 1);
        // owner: the first lane whose inclusive sum exceeds tt
        int j = 0;
#pragma unroll
        for (int step = kWave / 2; step > 0; step >>= 1)
            if (__shfl(incl, j + step - 1) <= tt) j += step;
        const uint32_t first = __shfl(incl, j) - __shfl(deg, j);
        const uint32_t base = __shfl(ob, j);
        const int32_t x = t < total ? load_idx(a.out_idx + base + (tt - first)) : -1;
        const uint32_t st = x >= 0 ? a.stamp[x] : 0xFFFFFFFFu;
        bool nw = false;
        if (st < a.sbase) {
            if (SPARSE) nw = atomicMax(&a.stamp[x], sv) < a.sbase;
            else a.stamp[x] = sv;
        }
        if (SPARSE) {
            const int cls = nw ? class_of_id(a, x) : 0;
            append_to_bins(nw, x, cls, a.ctl, a.bins, a.n_stride);
        }
    }
}

// Finish one row: Eq. 1, Delta r, writes; returns whether it must expand.
template <bool DF, bool F32>
__device__ __forceinline__ bool finish_row(const IterArgs &a, int32_t v, uint32_t cnt, double s, double rc,
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
    if (DF && dr > acc.ftol && a.xstamp[v] != a.sbase) {
        a.xstamp[v] = a.sbase;
        acc.c[2] += 1;
        acc.c[3] += oc;
        return true;
    }
    return false;
}

// One wave unit: 64/G rows of a class list (`list`), or of the id range
// starting at `id0` when `list` is NULL, G lanes per row.  LOOP (G = 1): the
// id range of rows whose only in-entry was the self-loop at load; few of
// them are marked, so their stamp is read first, and a row that has since
// gained in-edges is summed like any class-0 row.
template <int G, bool DF, bool F32, bool LOOP = false>
__device__ __forceinline__ void wave_unit(const IterArgs &a, const Hub &hub, const int32_t *list,
                                          uint32_t id0, uint32_t count, uint32_t first,
                                          bool check, bool sparse, Acc &acc)
{
    const int lane = lane_id();
    const int sub = lane & (G - 1);
    const uint32_t pos = first + lane / G;
    bool active = false;
    int32_t v = 0;
    uint32_t beg = 0, cnt = 0, oc = 1;
    double rc = 0.0;
    if (pos < count) {
        v = list ? list[pos] : (int32_t)(id0 + pos);
        active = true;
        if (LOOP) {
            if (DF && check) {
                const uint32_t st = a.stamp[v];
                active = st >= a.sbase && st <= a.sbase + (uint32_t)a.it;
            }
            if (active) {
                cnt = a.in_cnt[v];
                beg = a.in_beg[v];
                rc = a.Rc[v];
                oc = a.out_cnt[v];
            }
        } else {
            // the row's start, length, rank and out-degree are loaded with
            // its stamp, not after it: on the full schedule (dense mode)
            // only marked rows are processed, but waiting for the stamp
            // first would add a dependent load to every row (1.6% per call
            // on R-MAT scale 22)
            beg = a.in_beg[v];
            cnt = a.in_cnt[v];
            if (sub == 0) {
                rc = a.Rc[v];
                oc = a.out_cnt[v];
            }
            if (DF && check) {
                const uint32_t st = a.stamp[v];
                active = st >= a.sbase && st <= a.sbase + (uint32_t)a.it;
            }
        }
    }
    double s = 0.0;
    if (active) {
        if (cnt == 1) {
            // the self-loop is the only in-edge
            if (sub == 0) s = F32 ? (double)a.C32c[v] : a.Cc[v];
        } else if (LOOP) {
            // a self-loop row that has gained in-edges since the load: rare,
            // summed in index order by its lane (as gather_sum with G = 1)
            if (F32) {
                float ks = 0.0f, kc = 0.0f;
                for (uint32_t k = 0; k < cnt; k++) {
                    const float y = a.C32c[load_idx(a.in_idx + beg + k)] - kc;
                    const float t = ks + y;
                    kc = (t - ks) - y;
                    ks = t;
                }
                s = (double)ks - (double)kc;
            } else {
                for (uint32_t k = 0; k < cnt; k++) s += a.Cc[load_idx(a.in_idx + beg + k)];
            }
        } else {
            s = gather_sum<F32>(a, hub, a.in_idx + beg, sub, G, cnt);
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    bool expand = false;
    if (active && sub == 0) expand = finish_row<DF, F32>(a, v, cnt, s, rc, oc, acc);
    // Rows with fewer out-edges than a wave has lanes expand together, one
    // out-edge per lane and round; longer rows one at a time with the whole
    // wave and kUnroll loads in flight per lane.
    if (DF && __ballot(expand)) {
        const uint32_t sv = a.sbase + (uint32_t)a.it + 1;
        const bool small = expand && oc < (uint32_t)kWave;
        if (__ballot(small)) {
            const uint32_t deg = small ? oc : 0u;
            const uint32_t ob = small ? a.out_beg[v] : 0u;
            uint32_t incl = deg;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d);
                if (lane >= d) incl += y;
            }
            const uint32_t total = __shfl(incl, kWave - 1);
            if (sparse && !acc.plain) {
                expand_rows<true>(a, incl, deg, ob, total, sv);
            } else {
                if (sparse && lane == 0) a.ctl->force_dense = 1;
                expand_rows<false>(a, incl, deg, ob, total, sv);
            }
        }
        unsigned long long q = __ballot(expand && !small);
        while (q) {
            const int l = __ffsll((long long)q) - 1;
            const int32_t w = __shfl(v, l);
            const uint32_t wc = __shfl(oc, l);
            if (sparse && !acc.plain && !heavy_in_sparse(a, wc)) {
                mark_out_row<true>(a, w, lane, kWave, sv);
            } else {
                if (sparse && lane == 0) a.ctl->force_dense = 1;
                mark_out_row<false>(a, w, lane, kWave, sv);
            }
            q &= q - 1;
        }
    }
}

// One row of more than 1024 in-edges, the whole workgroup.  All threads
// call it with the same v.
template <bool DF, bool F32>
__device__ __forceinline__ void block_row(const IterArgs &a, const Hub &hub, int32_t v, bool valid,
                                 bool check, bool sparse, Acc &acc, double *red, int *flag)
{
    // A row of this class is summed by kBlock threads; a workgroup of more
    // threads sums one such row per kBlock of them (its sub-blocks), each
    // with the same partition and order as a kBlock workgroup.  Every
    // thread reaches the barriers, whether its sub-block has a row or not.
    const uint32_t t = threadIdx.x % kBlock;
    bool active = valid;
    if (active && DF && check) {
        const uint32_t st = a.stamp[v];
        active = st >= a.sbase && st <= a.sbase + (uint32_t)a.it;
    }
    uint32_t cnt = 0;
    if (active) {
        const uint32_t beg = a.in_beg[v];
        cnt = a.in_cnt[v];
        double s = gather_sum<F32>(a, hub, a.in_idx + beg, t, kBlock, cnt);
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (lane_id() == 0) red[t / kWave] = s;
    }
    __syncthreads();
    if (t == 0) {
        *flag = 0;
        if (active) {
            const double r = ((red[0] + red[1]) + red[2]) + red[3];
            *flag = finish_row<DF, F32>(a, v, cnt, r, a.Rc[v], a.out_cnt[v], acc) ? 1 : 0;
        }
    }
    __syncthreads();
    if (DF && *flag) {
        const uint32_t sv = a.sbase + (uint32_t)a.it + 1;
        if (sparse && !acc.plain && !heavy_in_sparse(a, a.out_cnt[v])) {
            mark_out_row<true>(a, v, t, kBlock, sv);
        } else {
            if (sparse && t == 0) a.ctl->force_dense = 1;
            mark_out_row<false>(a, v, t, kBlock, sv);
        }
    }
    __syncthreads();
}

// Fold a max and kCounters sums over a workgroup of W waves; thread 0 gets
// the result.  Waves fold with shuffles, then the wave results are combined
// in a fixed order.
template <int W = kWavesPerBlock>
__device__ __forceinline__ void block_fold(double &dr, double &rm, unsigned long long (&c)[kCounters],
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
        for (int w = 1; w < W; w++) {
            dr = fmax(dr, wdr[w]);
            rm = fmax(rm, wrm[w]);
#pragma unroll
            for (int j = 0; j < kCounters; j++) c[j] += wc[w][j];
        }
    }
    __syncthreads();
}

// Work of one iteration: per class, the list and its length; wave units
// of classes 5..0 and then of the self-loop-only rows (their own id
// range; class lists hold them in class 0), in that order; block units are
// the class-6 rows.
struct Plan {
    double ftol;                // frontier tolerance in effect
    uint32_t plain;             // Ctl::plain_marks
    uint32_t cnt[kBins];
    const int32_t *list[kBins]; // class lists (sparse), or NULL: the id range from id0
    uint32_t id0[kBins];
    uint32_t loop_cnt;          // the self-loop rows' id range (full schedule, DF)
    uint32_t loop_id0;
    uint32_t ustart[kBins];     // k < kBins - 1: class kBins - 2 - k; kBins - 1: loop rows
    uint32_t nwu, nbu;
};

__device__ __forceinline__ void make_plan(const IterArgs &a, const Ctl *ctl, bool sparse, bool df, int par,
                                 Plan &p)
{
    // a negative frontier tolerance asks for the call's adaptive choice
    p.ftol = a.ftol >= 0.0 ? a.ftol : ctl->ftol_used;
    p.plain = ctl->plain_marks;
    for (int b = 0; b < kBins; b++) {
        if (sparse) {
            p.cnt[b] = ctl->snap[par][b];
            p.list[b] = a.bins + (size_t)b * a.n_stride;
            p.id0[b] = 0;
        } else {
            // class b is the id range [cls[kBins - 1 - b], cls[kBins - b])
            p.cnt[b] = ctl->cls[kBins - b] - ctl->cls[kBins - 1 - b];
            p.list[b] = nullptr;
            p.id0[b] = ctl->cls[kBins - 1 - b];
        }
    }
    p.loop_cnt = sparse ? 0u : ctl->cls[kBins + 1] - ctl->cls[kBins];
    p.loop_id0 = ctl->cls[kBins];
    if (!df) {
        // every row is processed: class 0 and the self-loop rows are one
        // id range, walked as class 0
        p.cnt[0] += p.loop_cnt;
        p.loop_cnt = 0;
    }
    uint32_t acc = 0;
    for (int k = 0; k < kBins - 1; k++) {
        const int b = kBins - 2 - k;
        const uint32_t rows = kWave / group_of(b);
        p.ustart[k] = acc;
        acc += (p.cnt[b] + rows - 1) / rows;
    }
    p.ustart[kBins - 1] = acc;
    acc += (p.loop_cnt + kWave - 1) / kWave;
    p.nwu = acc;
    p.nbu = p.cnt[kBins - 1];
}

// Workgroups that have work in an iteration: 0 .. active-1.  With no work
// at all, workgroup 0 alone records the (empty) iteration.
template <int NW = kWavesPerBlock>
__device__ __forceinline__ uint32_t active_blocks(const Plan &p, uint32_t grid)
{
    constexpr uint32_t S = NW / kWavesPerBlock;    // rows of the block class at once
    const uint32_t wblocks = (p.nwu + NW - 1) / NW;
    return max(1u, max(min(grid, (p.nbu + S - 1) / S), min(grid, wblocks)));
}

// Shared memory of one workgroup of an iteration.
template <int NW = kWavesPerBlock>
struct IterSharedT {
    Plan plan;
    double red[NW];
    int flag[NW / kWavesPerBlock];
    double wdr[NW], wrm[NW];
    unsigned long long wc[NW][kCounters];
};
using IterShared = IterSharedT<>;

// Threads of the per-iteration fold.  Its time is the launch and one round
// trip to the slots, not the fold: 1024 threads (one round of loads for a
// full grid) were no faster on R-MAT scale 22 and cost ~3 us per iteration
// more on small frontiers, and loading the control-block fields beside the
// slots left it at 4.3 us.
#ifndef DFPR_FINAL_THREADS
#define DFPR_FINAL_THREADS 256
#endif
constexpr int kFinalThreads = DFPR_FINAL_THREADS;
constexpr int kFinalWaves = kFinalThreads / kWave;

// Shared memory of the per-iteration fold.
struct FinalShared {
    int copy;
    double wdr[kFinalWaves], wrm[kFinalWaves];
    unsigned long long wc[kFinalWaves][kCounters];
};

// One workgroup's share of an iteration of one graph: workgroup blk of the
// G workgroups given to the graph.  Its results are folded into slot
// blk mod kFoldSlots.
template <bool DF, bool F32, int NW = kWavesPerBlock>
__device__ __forceinline__ void iter_body(const IterArgs &a, uint32_t blk, uint32_t G,
                                 IterSharedT<NW> &sh, double *hub_lds = nullptr)
{
    const Ctl *ctl = a.ctl;
    if (ctl->done || (F32 && ctl->phase_end)) return;
    const int par = a.it & 1;
    const bool sparse = DF && !ctl->dense;
    const bool check = DF && !sparse;
    if (threadIdx.x == 0) make_plan(a, ctl, sparse, DF, par, sh.plan);
    __syncthreads();
    if (blk >= active_blocks<NW>(sh.plan, G)) return;
    const uint32_t nbu = sh.plan.nbu, nwu = sh.plan.nwu;
    // a sweep over the full schedule reads the hub contributions from LDS
    Hub hub{hub_lds, reinterpret_cast<const float *>(hub_lds), 0u};
    if (hub_lds && a.hub && !sparse) {
        hub.n = min(a.hub, (uint32_t)a.n);
        if (F32) {
            float *f = reinterpret_cast<float *>(hub_lds);
            for (uint32_t k = threadIdx.x; k < hub.n; k += NW * kWave) f[k] = a.C32c[k];
        } else {
            for (uint32_t k = threadIdx.x; k < hub.n; k += NW * kWave) hub_lds[k] = a.Cc[k];
        }
        __syncthreads();
    }

    Acc acc;
    acc.ftol = sh.plan.ftol;
    acc.plain = sh.plan.plain != 0;
    const int wave = threadIdx.x / kWave;
    auto run_unit = [&](uint32_t u, int k) {
        if (k == kBins - 1) {
            const uint32_t first = (u - sh.plan.ustart[k]) * kWave;
            wave_unit<1, DF, F32, true>(a, hub, nullptr, sh.plan.loop_id0, sh.plan.loop_cnt,
                                        first, check, sparse, acc);
            return;
        }
        const int b = kBins - 2 - k;
        const uint32_t first = (u - sh.plan.ustart[k]) * (kWave / group_of(b));
        const int32_t *list = sh.plan.list[b];
        const uint32_t id0 = sh.plan.id0[b];
        const uint32_t cnt = sh.plan.cnt[b];
        switch (b) {
        case 0: wave_unit<1, DF, F32>(a, hub, list, id0, cnt, first, check, sparse, acc); break;
        case 1: wave_unit<2, DF, F32>(a, hub, list, id0, cnt, first, check, sparse, acc); break;
        case 2: wave_unit<4, DF, F32>(a, hub, list, id0, cnt, first, check, sparse, acc); break;
        case 3: wave_unit<8, DF, F32>(a, hub, list, id0, cnt, first, check, sparse, acc); break;
        case 4: wave_unit<32, DF, F32>(a, hub, list, id0, cnt, first, check, sparse, acc); break;
        default: wave_unit<64, DF, F32>(a, hub, list, id0, cnt, first, check, sparse, acc); break;
        }
    };
    const int32_t *blist = sh.plan.list[kBins - 1];
    constexpr uint32_t S = NW / kWavesPerBlock;     // sub-blocks of kBlock threads
    const uint32_t sub = threadIdx.x / kBlock;
    for (uint32_t u0 = blk * S; u0 < nbu; u0 += G * S) {
        const uint32_t u = u0 + sub;
        const bool valid = u < nbu;
        const int32_t v = !valid ? 0 : blist ? blist[u] : (int32_t)(sh.plan.id0[kBins - 1] + u);
        block_row<DF, F32>(a, hub, v, valid, check, sparse, acc, sh.red + sub * kWavesPerBlock,
                           sh.flag + sub);
    }
    for (uint32_t u = blk * NW + wave; u < nwu; u += G * NW) {
        int k = 0;
        while (k + 1 < kBins && u >= sh.plan.ustart[k + 1]) k++;
        run_unit(u, k);
    }

    double dr = acc.dr_max, rm = acc.r_max;
    unsigned long long c[kCounters];
#pragma unroll
    for (int j = 0; j < kCounters; j++) c[j] = acc.c[j];
    block_fold<NW>(dr, rm, c, sh.wdr, sh.wrm, sh.wc);
    if (threadIdx.x == 0) {
        // non-negative doubles order like their bit patterns
        const uint32_t slot = blk % kFoldSlots;
        atomicMax(reinterpret_cast<unsigned long long *>(a.dr_part) + slot,
                  (unsigned long long)__double_as_longlong(dr));
        atomicMax(reinterpret_cast<unsigned long long *>(a.rmax_part) + slot,
                  (unsigned long long)__double_as_longlong(rm));
#pragma unroll
        for (int j = 0; j < kCounters; j++)
            if (c[j]) atomicAdd(&a.cnt_part[slot * kCounters + j], c[j]);
    }
}

// After each iteration (one workgroup): fold the slots the iteration's
// workgroups left, decide convergence or the cap, and prepare the next
// iteration.  The launch boundary orders it after k_iter.
// In the FP32 phase of the precision form, reaching tol or the FP32
// resolution of the ranks ends the phase instead of the call.
// The control block goes to the host mirror when `last` (the last launch
// the host queued before it next waits) or when this step ends the call or
// the phase: later launches then return at once.
__device__ __forceinline__ void final_body(const IterArgs &a, bool df, bool f32, FinalShared &sh, bool last)
{
    Ctl *ctl = a.ctl;
    if (ctl->done || (f32 && ctl->phase_end)) return;
    const int par = a.it & 1;
    const bool sparse = df && !ctl->dense;
    double dr = 0.0, rm = 0.0;
    unsigned long long c[kCounters] = {0, 0, 0, 0};
    // each thread reads its slots and clears them for the next iteration
    for (uint32_t i = threadIdx.x; i < (uint32_t)kFoldSlots; i += kFinalThreads) {
        dr = fmax(dr, a.dr_part[i]);
        rm = fmax(rm, a.rmax_part[i]);
#pragma unroll
        for (int j = 0; j < kCounters; j++) c[j] += a.cnt_part[i * kCounters + j];
        a.dr_part[i] = 0.0;
        a.rmax_part[i] = 0.0;
#pragma unroll
        for (int j = 0; j < kCounters; j++) a.cnt_part[i * kCounters + j] = 0ull;
    }
    block_fold<kFinalWaves>(dr, rm, c, sh.wdr, sh.wrm, sh.wc);
    if (threadIdx.x == 0) {
        ctl->verts += c[0];
        ctl->edges += c[1];
        ctl->xverts += c[2];
        ctl->xedges += c[3];
        ctl->iterations = a.it + 1;
        ctl->final_linf = dr;
        ctl->final_rmax = rm;
        if (sparse) {
            unsigned long long before = 0, after = 0;
            for (int b = 0; b < kBins; b++) {
                const uint32_t l = ctl->live[b];
                before += ctl->snap[par][b];
                after += l;
                ctl->snap[par ^ 1][b] = l;
            }
            ctl->marked += after - before;
            if (after > a.sparse_limit || ctl->force_dense) ctl->dense = 1;
        }
        if (f32) {
            // FP32 contributions carry a relative rounding error of 2^-24;
            // changes below about 2^-22 of the largest rank are noise.  A
            // Delta R that stops falling counts as a stall only near that
            // floor (early on it can rise while the frontier grows).
            const double floor32 = rm * 0x1p-22;
            const bool stalled = ctl->phase_iters >= 3 && dr >= 0.97 * ctl->prev_linf &&
                                 dr <= rm * 0x1p-16;
            ctl->phase_iters += 1;
            if (dr <= a.tol || dr <= floor32 || stalled) ctl->phase_end = 1;
            if (a.it + 1 >= a.max_iters) ctl->done = 1;
        } else {
            const bool conv = dr <= a.tol;
            if (conv) ctl->converged = 1;
            if (conv || a.it + 1 >= a.max_iters) ctl->done = 1;
        }
        ctl->prev_linf = dr;
        sh.copy = a.mirror && (last || ctl->done || (f32 && ctl->phase_end));
    }
    __syncthreads();
    if (sh.copy && threadIdx.x < kWave) {
        // one wave copies the words of the block (thread 0's updates are
        // visible after the barrier)
        constexpr int words = (int)(sizeof(Ctl) / 4);
        const volatile uint32_t *src = reinterpret_cast<const volatile uint32_t *>(ctl);
        uint32_t *dst = reinterpret_cast<uint32_t *>(a.mirror);
        for (int i = threadIdx.x; i < words; i += kWave) dst[i] = src[i];
    }
}



}  // namespace dfpr

namespace dfpr {

// Host helpers of rank.hip shared with the serving loop (serve.hip).
IterArgs iter_args(dfpr_graph *g, const dfpr_params &p, uint32_t sbase);
int check_params(const dfpr_params *p, dfpr_params &out);
int df_begin(dfpr_graph *g, const dfpr_params &p, int64_t nd, const int32_t *bds,
             const int32_t *bdd, int64_t ni, const int32_t *bis, const int32_t *bid,
             const double *prev, int prev_dev, uint32_t *sbase_out, int32_t *lists = nullptr);
// A Dynamic Frontier call on device arrays whose batch is staged in
// `staging` (4 (nd + ni) ints) instead of the library's buffer.
int df_device_staged(dfpr_graph *g, const dfpr_params *pp, int64_t nd, const int32_t *ds,
                     const int32_t *dd, int64_t ni, const int32_t *is, const int32_t *id,
                     const double *prev, double *ranks_out, dfpr_stats *st, int32_t *staging);
int df_phase_end(dfpr_graph *g, int res, bool call_done);
int df_finish(dfpr_graph *g, uint32_t sbase, int res, int32_t iters);

}  // namespace dfpr
