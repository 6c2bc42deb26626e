// Rank engines: Static, Naive-dynamic and Dynamic Frontier PageRank.
//
// One iteration of every engine is one launch of k_iter, which
//   - pulls Eq. 1 for the rows of the iteration: every vertex (Static,
//     Naive-dynamic) or the affected vertices (Dynamic Frontier);
//   - computes Delta r = |r - R[v]| and the L-inf maximum;
//   - (Dynamic Frontier) marks the out-neighbours of every row whose rank
//     moved by more than frontier_tol;
// followed by a one-workgroup launch of k_final that folds the slots the
// workgroups folded their results into and decides convergence
// (Delta R <= tol) or the iteration cap.
// The host enqueues iterations in chunks and reads the stop flag between
// chunks; launches issued after the stop flag is set return at once.
//
// Work layout.  Rows are split by in-degree into classes; a class-b row is
// reduced by group_of(b) lanes of one wave (1, 2, 4, 8, 32 or 64 lanes) or,
// above 1024 in-edges, by a whole workgroup.  Internal ids follow
// decreasing in-degree at load, so each class is an id range, and a row
// keeps the class of its id for the life of the graph (Ctl::cls).
// Rows whose only in-entry was the self-loop form the last range.  Each
// lane loads kUnroll indices and then kUnroll contributions per round, so
// that many loads are in flight per wave.  Each lane sums its strided share
// of a row in order and the group folds the partial sums with a fixed
// butterfly, so the sum of a row depends on nothing but the row and its id.
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
// lists pass a size limit, iterations walk every class's id range and skip
// rows whose stamp is out of range (dense mode, the "full schedule"); marks
// are then plain stores.  Expansions that would append more than the lists
// take (a row with a very long out-row, or a first frontier whose out-rows
// together pass the limit) also mark with plain stores, and the call walks
// the full schedule from the next iteration on.  Neither walk needs
// rebuilding when a batch changes in-degrees.
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
#include "iter.h"

namespace dfpr {


template <bool DF, bool F32>
__global__ __launch_bounds__(kBlock, DFPR_ITER_WAVES_PER_SIMD) void k_iter(IterArgs a)
{
    __shared__ IterShared sh;
#if DFPR_HUB
    __shared__ double hub[kHubRows];
    iter_body<DF, F32>(a, blockIdx.x, gridDim.x, sh, hub);
#else
    iter_body<DF, F32>(a, blockIdx.x, gridDim.x, sh);
#endif
}

// The full schedule in wide workgroups: more waves per workgroup, fewer
// workgroups per CU, the same 6 waves per SIMD as k_iter, and one larger
// LDS copy of the first contributions per workgroup instead of one of
// kHubRows per four waves.  Static and Naive-dynamic sweeps (Eq. 1 over
// every vertex) use 12 waves and 9216 entries (two workgroups per CU; about
// 34% of the gathers on R-MAT scale 22 read LDS instead of 18%, 4% less time
// per sweep).  Dynamic Frontier iterations on the full schedule use 8 waves
// and 6144 entries (three per CU; 12 waves left that kernel at the 80-VGPR
// cap with a spill and no gain, 8 give 1% per call), or 12288 FP32 entries
// in the FP32 phase of the precision form (2.5% per call at R-MAT scale 24).
// Results are bitwise those of k_iter: block-class rows keep their kBlock
// partition (see block_row).
#ifndef DFPR_WIDE
#define DFPR_WIDE 1
#endif
#ifndef DFPR_WIDE_HUB
#define DFPR_WIDE_HUB 9216
#endif
#ifndef DFPR_WIDE_F32_MUL
#define DFPR_WIDE_F32_MUL 2
#endif
#ifndef DFPR_WIDE_DF_HUB
#define DFPR_WIDE_DF_HUB 6144
#endif
constexpr int kWideWaves = 12, kWideDfWaves = 8;
constexpr uint32_t kWideHub = DFPR_WIDE_HUB, kWideDfHub = DFPR_WIDE_DF_HUB;

template <bool DF, bool F32, int NW, uint32_t HUB>
__global__ __launch_bounds__(NW * kWave, 6) void k_iter_wide(IterArgs a)
{
    __shared__ IterSharedT<NW> sh;
    __shared__ double hub[HUB];
    iter_body<DF, F32, NW>(a, blockIdx.x, gridDim.x, sh, hub);
}

// After each iteration (one workgroup): fold the slots the iteration's
// workgroups left, decide convergence or the cap, and prepare the next
// iteration.  The launch boundary orders it after k_iter.
__global__ __launch_bounds__(kFinalThreads) void k_final(IterArgs a, int df, int f32, int last)
{
    __shared__ FinalShared sh;
    final_body(a, df != 0, f32 != 0, sh, last != 0);
}

// ---------------------------------------------------------------------------
// small-frontier loop
// ---------------------------------------------------------------------------
// While the class lists hold few rows, an iteration's two launches and their
// kernel boundaries cost more than its rows.  k_loop runs the iterations of
// Algorithm 1's loop inside one cooperative launch of a few workgroups
// instead: the rows of an iteration are spread over the workgroups exactly as
// in k_iter, a grid barrier separates the pull from the fold (workgroup 0
// runs final_body), and a second barrier publishes the new control block.
// The launch hands back to the host loop when the call or the FP32 phase
// ends, when an iteration has more rows than `limit` or the call moves to
// the full schedule, or after kLoopChunk iterations.  Every row is summed
// as in k_iter, so the ranks do not depend on which loop ran an iteration.
#ifndef DFPR_LOOP_GRID
#define DFPR_LOOP_GRID 64
#endif
#ifndef DFPR_LOOP_ROWS
#define DFPR_LOOP_ROWS 16384
#endif
constexpr int kLoopGrid = DFPR_LOOP_GRID;        // workgroups of the small-frontier loop
constexpr uint32_t kLoopRows = DFPR_LOOP_ROWS;   // most rows of an iteration it runs
constexpr uint32_t kSpinLimit = 1u << 22;        // polls of a grid barrier before it gives up

struct LoopArgs {
    double *R[2], *C[2];
    float *C32[2];
    int32_t base;       // buffer that iteration it0 reads
    int32_t it0;        // first iteration of the phase (buffer parity)
    int32_t it_start;   // first iteration of this launch
    uint32_t limit;     // rows of an iteration above which the launch hands over
    int32_t bar;        // barrier counter of the control block
};

// All workgroups of the launch meet here.  The counter only grows: the
// k-th barrier of a launch waits for k * gridDim.x arrivals.  Releases and
// acquires are at agent scope, so the rows, marks and lists one workgroup
// wrote are visible to all after it.  Returns false if the others did not
// arrive within kSpinLimit polls (every workgroup then leaves the loop).
__device__ inline bool grid_barrier(uint32_t *count, uint32_t target, int *s_ok)
{
    __syncthreads();
    if (gridDim.x == 1) return true;   // one workgroup: its barrier orders everything
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        int ok = 1;
        while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins == kSpinLimit) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

template <bool F32>
__global__ __launch_bounds__(kBlock) void k_loop(IterArgs a, LoopArgs L)
{
    __shared__ IterShared sh;
    __shared__ FinalShared fsh;
    __shared__ int s_go, s_ok;
    Ctl *ctl = a.ctl;
    uint32_t *bar = &ctl->bar[L.bar];
    const uint32_t G = gridDim.x;
    uint32_t passed = 0;
    bool failed = false;
    for (int k = 0; k < kLoopChunk; k++) {
        const int i = L.it_start + k;
        if (threadIdx.x == 0) {
            // every workgroup reads the same state: it was written before
            // the last barrier (or by an earlier launch)
            uint32_t rows = 0;
            for (int b = 0; b < kBins; b++) rows += ctl->snap[i & 1][b];
            s_go = !(ctl->done || (F32 && ctl->phase_end) || ctl->dense || ctl->loop_fail) &&
                   rows <= L.limit && i < a.max_iters;
        }
        __syncthreads();
        if (!s_go) break;
        const int src = L.base ^ ((i - L.it0) & 1);
        IterArgs ai = a;
        ai.it = i;
        ai.Rc = L.R[src];
        ai.Cc = L.C[src];
        ai.Rn = L.R[src ^ 1];
        ai.Cn = L.C[src ^ 1];
        ai.C32c = L.C32[src];
        ai.C32n = L.C32[src ^ 1];
        iter_body<true, F32>(ai, blockIdx.x, G, sh);
        if (!grid_barrier(bar, ++passed * G, &s_ok)) {
            failed = true;
            break;
        }
        if (blockIdx.x == 0) final_body(ai, true, F32, fsh, false);
        if (!grid_barrier(bar, ++passed * G, &s_ok)) {
            failed = true;
            break;
        }
    }
    if (failed && threadIdx.x == 0) {
        __hip_atomic_store(&ctl->loop_fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        // the state for the host (workgroup 0 wrote the last fold itself)
        __syncthreads();
        constexpr int words = (int)(sizeof(Ctl) / 4);
        const volatile uint32_t *src = reinterpret_cast<const volatile uint32_t *>(ctl);
        uint32_t *dst = reinterpret_cast<uint32_t *>(a.mirror);
        for (int w = threadIdx.x; w < words; w += kBlock) dst[w] = src[w];
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
        ctl->force_dense = 0;
        ctl->plain_marks = 0;
        ctl->phase_end = 0;
        ctl->phase_iters = 0;
        ctl->prev_linf = 0.0;
        ctl->renorm_scale = 1.0;
        ctl->iterations = 0;
        ctl->converged = 0;
        ctl->final_linf = 0.0;
        ctl->final_rmax = 0.0;
        ctl->edges = ctl->verts = 0;
        ctl->xverts = ctl->xedges = ctl->marked = 0;
        ctl->affected0 = ctl->affected = 0;
        ctl->err = 0;
        ctl->mk_light = ctl->mk_heavy = 0;
        ctl->reach = 0;
        for (int k = 0; k < 3; k++) ctl->qn[k] = ctl->qhn[k] = 0;
        ctl->bar[0] = ctl->bar[1] = 0;
        ctl->loop_fail = 0;
        ctl->reach0 = 0;
        ctl->ftol_used = 0.0;
    }
}

// Freeze the lists built by the marking as iteration 0's snapshot and pick
// the walk of the first iteration.
// Adaptive frontier tolerance (the paper leaves the choice of tau_f by the
// nature of the batch to future work, Section 5.2.4 and the Conclusion).
// The initial marking measures how fast the frontier can grow: the mean
// out-degree g of the vertices it marked.  Mesh-like neighbourhoods (g <= 8)
// let the frontier creep outward over many iterations of changes far below
// tol, so expansion stops early (tau_f = tol/10); hub-rich ones (g > 64)
// reach most of the graph within a few iterations whatever tau_f is, so the
// accurate tol/1e5 costs little; the steps between take tol/100 ... tol/1e4.
// Integer comparisons only, so the choice is exact.
__host__ __device__ inline int adaptive_ftol_exponent(unsigned long long marked,
                                                      unsigned long long out_edges)
{
    if (marked == 0) return 5;
    return out_edges <= 8 * marked ? 1 : out_edges <= 16 * marked ? 2
         : out_edges <= 32 * marked ? 3 : out_edges <= 64 * marked ? 4 : 5;
}

__global__ void k_snap(Ctl *ctl, int32_t max_iters, uint32_t sparse_limit, int dense, Ctl *mirror,
                       double tol, double ftol)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (ftol >= 0.0) {
            ctl->ftol_used = ftol;
        } else {
            const double p10[6] = {1.0, 1e1, 1e2, 1e3, 1e4, 1e5};
            ctl->ftol_used = tol / p10[adaptive_ftol_exponent(ctl->affected0, ctl->reach0)];
        }
        unsigned long long tot = 0;
        for (int b = 0; b < kBins; b++) {
            ctl->snap[0][b] = ctl->live[b];
            tot += ctl->live[b];
        }
        ctl->dense = (dense || ctl->dense || tot > sparse_limit) ? 1 : 0;
        // a first frontier with more out-edges than the class lists take
        // would append most of them in its first expansions, one list
        // atomic per wave and round on counters that share a cache line;
        // its expansions mark with plain stores instead, and the call walks
        // the full schedule from the next iteration on
        ctl->plain_marks = ctl->reach0 > sparse_limit ? 1 : 0;
        ctl->done = (ctl->err || max_iters <= 0) ? 1 : 0;
        if (mirror) __builtin_memcpy(mirror, ctl, sizeof(Ctl));
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

// Initial marking (Section 4.1.1, Algorithm 1): every batch edge (u, v)
// marks G^t.out(u), and a deletion also marks v, which was in
// G^{t-1}.out(u).  Marks are stamps equal to the call's base.  A source
// whose out-row has been scanned gets its expansion stamp, so it never
// scans that row again in this call.
//
// Claim pass, one thread per batch entry: the first entry of each distinct
// source claims it through its expansion stamp; claimed sources go to a
// light list (out-row scanned by one wave) or a heavy list (scanned by the
// whole grid in workgroup-sized chunks), and their out-degrees are summed.
constexpr uint32_t kHeavyRow = 2048;   // out-rows longer than this use the grid
constexpr uint32_t kHeavySeg = 2048;   // heavy vertices whose chunk offsets sit in LDS at once

struct HeavyShared {
    uint32_t pre[kHeavySeg + 1];       // chunk offsets of a segment of heavy vertices
    uint32_t part[kBlock];
};

// Walk the out-rows of the heavy vertices list[0 .. nh) in chunks of kBlock
// out-edges: chunk c of the concatenated rows goes to workgroup
// c mod gridDim.x.  Each workgroup finds the vertex of a chunk by binary
// search over the chunk offsets, which it builds in LDS for up to
// kHeavySeg vertices at a time, so no workgroup walks the list serially.
// visit(x) is called by every thread of the workgroup with the same trip
// count (x < 0: no vertex).
template <class F>
__device__ inline void walk_heavy(const IterArgs &a, const int32_t *list, uint32_t nh,
                                  HeavyShared &sh, F &&visit)
{
    constexpr uint32_t per = kHeavySeg / kBlock;
    for (uint32_t h0 = 0; h0 < nh; h0 += kHeavySeg) {
        const uint32_t seg = min(kHeavySeg, nh - h0);
        // per thread: chunk counts of `per` consecutive vertices, then a scan
        // of the thread totals
        uint32_t cnt[per], tot = 0;
#pragma unroll
        for (uint32_t j = 0; j < per; j++) {
            const uint32_t i = threadIdx.x * per + j;
            cnt[j] = i < seg ? (a.out_cnt[list[h0 + i]] + kBlock - 1) / kBlock : 0u;
            tot += cnt[j];
        }
        sh.part[threadIdx.x] = tot;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            const uint32_t t = threadIdx.x >= (uint32_t)o ? sh.part[threadIdx.x - o] : 0u;
            __syncthreads();
            sh.part[threadIdx.x] += t;
            __syncthreads();
        }
        uint32_t run = sh.part[threadIdx.x] - tot;
#pragma unroll
        for (uint32_t j = 0; j < per; j++) {
            const uint32_t i = threadIdx.x * per + j;
            if (i < seg) sh.pre[i] = run;
            run += cnt[j];
        }
        if (threadIdx.x == kBlock - 1) sh.pre[seg] = sh.part[kBlock - 1];
        __syncthreads();
        const uint32_t total = sh.pre[seg];
        for (uint32_t c = blockIdx.x; c < total; c += gridDim.x) {
            uint32_t lo = 0, hi = seg;      // last h with pre[h] <= c
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) / 2;
                if (sh.pre[mid] <= c) lo = mid;
                else hi = mid;
            }
            const int32_t u = list[h0 + lo];
            const uint32_t k = (c - sh.pre[lo]) * kBlock + threadIdx.x;
            const uint32_t oc = a.out_cnt[u];
            visit(k < oc ? a.out_idx[a.out_beg[u] + k] : -1);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_mark_claim(IterArgs a, int64_t nd, const int32_t *ds,
                                                       int64_t ni, const int32_t *is,
                                                       int32_t *light, int32_t *heavy)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t u = -1;
    if (i < nd + ni) u = i < nd ? ds[i] : is[i - nd];
    bool take = false;
    uint32_t oc = 0;
    if (u >= 0 && u < a.n && a.xstamp[u] != a.sbase) {
        take = atomicMax(&a.xstamp[u], a.sbase) < a.sbase;
        if (take) oc = a.out_cnt[u];
    }
    const bool big = take && oc > kHeavyRow;
    const int lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long ml = __ballot(take && !big), mh = __ballot(big);
    unsigned long long r = oc;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) r += __shfl_xor(r, off, kWave);
    uint32_t bl = 0, bh = 0;
    if (lane == 0) {
        if (ml) bl = atomicAdd(&a.ctl->mk_light, (uint32_t)__popcll(ml));
        if (mh) bh = atomicAdd(&a.ctl->mk_heavy, (uint32_t)__popcll(mh));
        if (r) atomicAdd(&a.ctl->reach, r);
    }
    bl = __shfl(bl, 0);
    bh = __shfl(bh, 0);
    if (take && !big) light[bl + __popcll(ml & below)] = u;
    if (big) heavy[bh + __popcll(mh & below)] = u;
}

// Mark x (x < 0: no vertex).  Every lane of the wave calls it.  Lane 0
// counts the new marks in `mine` and, in `deg`, their out-edges.
__device__ inline void mark_one(const IterArgs &a, int32_t x, bool append,
                                unsigned long long &mine, unsigned long long &deg)
{
    bool nw = false;
    if (x >= 0 && a.stamp[x] < a.sbase) nw = atomicMax(&a.stamp[x], a.sbase) < a.sbase;
    const unsigned long long m = __ballot(nw);
    unsigned long long d = nw ? a.out_cnt[x] : 0u;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) d += __shfl_xor(d, off, kWave);
    if (lane_id() == 0) {
        mine += __popcll(m);
        deg += d;
    }
    if (append) {
        const int cls = nw ? class_of_id(a, x) : 0;
        append_to_bins(nw, x, cls, a.ctl, a.bins, a.n_stride);
    }
}

// Marking pass: deletion targets, then light sources one wave each, then
// heavy sources in chunks of kBlock out-edges spread over the grid.  The
// class lists are filled (sparse mode) unless `dense` is set or the claimed
// sources reach more vertices than the sparse limit; the decision goes to
// the control block for the iterations.  Every loop bound is uniform
// within a wave.
__global__ __launch_bounds__(kBlock) void k_mark_initial(IterArgs a, int64_t nd, const int32_t *dd,
                                                         const int32_t *light,
                                                         const int32_t *heavy, int dense)
{
    __shared__ unsigned long long s_new, s_deg;
    Ctl *ctl = a.ctl;
    if (ctl->err) return;
    const bool dn = dense || ctl->reach + (unsigned long long)nd > a.sparse_limit;
    const bool append = !dn;
    if (blockIdx.x == 0 && threadIdx.x == 0 && dn) ctl->dense = 1;
    if (threadIdx.x == 0) s_new = s_deg = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    unsigned long long mine = 0, mdeg = 0;
    for (int64_t b0 = wave * kWave; b0 < nd; b0 += waves * kWave) {
        const int64_t i = b0 + lane;
        mark_one(a, i < nd ? dd[i] : -1, append, mine, mdeg);
    }
    const uint32_t nl = ctl->mk_light, nh = ctl->mk_heavy;
    for (int64_t w = wave; w < nl; w += waves) {
        const int32_t u = light[w];
        const uint32_t ob = a.out_beg[u], oc = a.out_cnt[u];
        for (uint32_t kb = 0; kb < oc; kb += kWave) {
            const uint32_t k = kb + lane;
            mark_one(a, k < oc ? a.out_idx[ob + k] : -1, append, mine, mdeg);
        }
    }
    __shared__ HeavyShared hs;
    walk_heavy(a, heavy, nh, hs, [&](int32_t x) { mark_one(a, x, append, mine, mdeg); });
    if (lane == 0 && mine) {
        atomicAdd(&s_new, mine);
        atomicAdd(&s_deg, mdeg);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_new) {
        atomicAdd(&ctl->affected0, s_new);
        atomicAdd(&ctl->reach0, s_deg);
    }
}

// Dynamic Traversal (Section 3.3.2): every vertex reachable from the
// source of a batch edge in G^{t-1} or in G^t is affected.  Every deleted
// edge leaves a batch source, so the vertices reachable in either graph are
// those reachable along G^t's out-edges from the batch sources and the
// deletion targets.  A level-synchronous breadth-first search claims each
// vertex once through its stamp (the call's base, so that it is processed
// from the first iteration) and appends it to the next level's queue and,
// with `append`, to its class list.  Vertices with more than kHeavyRow
// out-edges go to a separate queue whose out-rows the whole grid walks in
// workgroup-sized chunks; the others are walked by waves, 64 at a time.
// Three queues (of each kind) rotate: level L reads queue L mod 3, fills
// queue L+1 mod 3 and clears the lengths of queue L+2 mod 3.

struct BfsQueues {
    const int32_t *in, *hin;          // this level: light and heavy vertices
    const uint32_t *nin, *nhin;
    int32_t *out, *hout;              // next level
    uint32_t *nout, *nhout;
    uint32_t *clear, *hclear;         // the level after next
};

// Every lane of the wave calls it; x < 0 claims nothing.
__device__ inline void bfs_claim(const IterArgs &a, int32_t x, const BfsQueues &q, bool append,
                                 unsigned long long &mine)
{
    bool nw = false;
    if (x >= 0 && a.stamp[x] < a.sbase) nw = atomicMax(&a.stamp[x], a.sbase) < a.sbase;
    const bool big = nw && a.out_cnt[x] > kHeavyRow;
    const unsigned long long ml = __ballot(nw && !big), mh = __ballot(big);
    const int lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    if (ml | mh) {
        uint32_t bl = 0, bh = 0;
        if (lane == 0) {
            if (ml) bl = atomicAdd(q.nout, (uint32_t)__popcll(ml));
            if (mh) bh = atomicAdd(q.nhout, (uint32_t)__popcll(mh));
            mine += __popcll(ml | mh);
        }
        bl = __shfl(bl, 0);
        bh = __shfl(bh, 0);
        if (nw && !big) q.out[bl + __popcll(ml & below)] = x;
        if (big) q.hout[bh + __popcll(mh & below)] = x;
    }
    if (append) {
        const int cls = nw ? class_of_id(a, x) : 0;
        append_to_bins(nw, x, cls, a.ctl, a.bins, a.n_stride);
    }
}

__global__ __launch_bounds__(kBlock) void k_bfs_seed(IterArgs a, int64_t nd, const int32_t *ds,
                                                     const int32_t *dd, int64_t ni,
                                                     const int32_t *is, BfsQueues q, int append)
{
    __shared__ unsigned long long s_new;
    if (a.ctl->err) return;
    if (threadIdx.x == 0) s_new = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    unsigned long long mine = 0;
    for (int64_t b0 = wave * kWave; b0 < nd + ni; b0 += waves * kWave) {
        const int64_t i = b0 + lane;
        const int32_t u = i < nd + ni ? (i < nd ? ds[i] : is[i - nd]) : -1;
        bfs_claim(a, u, q, append != 0, mine);
        bfs_claim(a, i < nd ? dd[i] : -1, q, append != 0, mine);
    }
    if (lane == 0 && mine) atomicAdd(&s_new, mine);
    __syncthreads();
    if (threadIdx.x == 0 && s_new) atomicAdd(&a.ctl->affected0, s_new);
}

// One level.  Light vertices: each wave takes 64 and walks their out-edges
// together, one out-edge per lane and round.  Heavy vertices: every
// workgroup takes chunks of kBlock out-edges of each of them.
__global__ __launch_bounds__(kBlock) void k_bfs_level(IterArgs a, BfsQueues q, int append)
{
    __shared__ unsigned long long s_new;
    if (a.ctl->err) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *q.clear = 0;
        *q.hclear = 0;
    }
    const uint32_t nin = *q.nin, nh = *q.nhin;
    if (threadIdx.x == 0) s_new = 0;
    __syncthreads();
    const int lane = lane_id();
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    unsigned long long mine = 0;
    for (int64_t b0 = wave * kWave; b0 < nin; b0 += waves * kWave) {
        const int64_t i = b0 + lane;
        const int32_t x = i < nin ? q.in[i] : -1;
        const uint32_t deg = x >= 0 ? a.out_cnt[x] : 0u;
        const uint32_t ob = x >= 0 ? a.out_beg[x] : 0u;
        uint32_t incl = deg;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        const uint32_t total = __shfl(incl, kWave - 1);
        for (uint32_t t0 = 0; t0 < total; t0 += kWave) {
            const uint32_t t = t0 + lane;
            const uint32_t tt = min(t, total - 1);
            int j = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1)
                if (__shfl(incl, j + step - 1) <= tt) j += step;
            const uint32_t first = __shfl(incl, j) - __shfl(deg, j);
            const uint32_t base = __shfl(ob, j);
            const int32_t y = t < total ? a.out_idx[base + (tt - first)] : -1;
            bfs_claim(a, y, q, append != 0, mine);
        }
    }
    __shared__ HeavyShared hs;
    walk_heavy(a, q.hin, nh, hs, [&](int32_t x) { bfs_claim(a, x, q, append != 0, mine); });
    if (lane == 0 && mine) atomicAdd(&s_new, mine);
    __syncthreads();
    if (threadIdx.x == 0 && s_new) atomicAdd(&a.ctl->affected0, s_new);
}

// End of a Dynamic Frontier call: copy the rows processed in this call from
// the result buffer into the other buffer and count the marked vertices.
// A call that stayed on the class lists visits the listed vertices (every
// mark of the call was appended); otherwise all vertices by stamp.
__global__ __launch_bounds__(kBlock) void k_finish(int32_t n, const uint32_t *stamp, uint32_t lo,
                                                   uint32_t hi, const double *Rres, double *Roth,
                                                   const double *Cres, double *Coth, Ctl *ctl,
                                                   const int32_t *bins, int32_t n_stride)
{
    __shared__ unsigned long long s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned long long mine = 0;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    if (!ctl->dense) {
        uint32_t len[kBins];
        int64_t tot = 0;
        for (int b = 0; b < kBins; b++) {
            len[b] = ctl->live[b];
            tot += len[b];
        }
        for (int64_t t = t0; t < tot; t += step) {
            int b = 0;
            int64_t r = t;
            while (r >= len[b]) r -= len[b++];
            const int32_t v = bins[(int64_t)b * n_stride + r];
            mine++;
            Roth[v] = Rres[v];
            Coth[v] = Cres[v];
        }
    } else {
        for (int64_t v = t0; v < n; v += step) {
            const uint32_t st = stamp[v];
            if (st >= lo && st <= hi) {
                mine++;
                Roth[v] = Rres[v];
                Coth[v] = Cres[v];
            }
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

// Both passes of the initial marking on the graph's stream.  The batch
// arrays are staged in device memory; `lists` has room for the two source
// lists (2 (nd + ni) entries).
static void launch_initial_marking(dfpr_graph *g, const IterArgs &a, int64_t nd,
                                   const int32_t *ds, const int32_t *dd, int64_t ni,
                                   const int32_t *is, int dense, int32_t *lists)
{
    int32_t *light = lists;
    int32_t *heavy = light + (nd + ni);
    k_mark_claim<<<blocks_for(nd + ni), kBlock, 0, g->stream>>>(a, nd, ds, ni, is, light, heavy);
    const int64_t waves = std::max<int64_t>(nd + ni, 1024);
    k_mark_initial<<<(unsigned)std::min<int64_t>(blocks_for(waves * kWave), 2048), kBlock, 0,
                     g->stream>>>(a, nd, dd, light, heavy, dense);
}


// The control block to its host copy (coherent pinned memory) by one wave.
// A copy-engine transfer of these few hundred bytes occupies the queue for
// ~20 us; a one-wave kernel takes a few.
__global__ __launch_bounds__(kWave) void k_ctl_to_host(const Ctl *ctl, Ctl *host)
{
    static_assert(sizeof(Ctl) % 4 == 0, "the control block is copied in 4-byte words");
    constexpr int words = (int)(sizeof(Ctl) / 4);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(ctl);
    uint32_t *dst = reinterpret_cast<uint32_t *>(host);
    for (int i = threadIdx.x; i < words; i += kWave) dst[i] = src[i];
}

int ctl_to_host(dfpr_graph *g)
{
    k_ctl_to_host<<<1, kWave, 0, g->stream>>>(g->ctl, g->ctl_host);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
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

int check_params(const dfpr_params *p, dfpr_params &out)
{
    if (p) out = *p;
    else dfpr_params_default(&out);
    if (!(out.alpha >= 0.0 && out.alpha < 1.0) || !(out.tol >= 0.0) ||
        std::isnan(out.frontier_tol) || out.max_iters < 0 || out.max_iters > 100000 ||
        (out.precision != DFPR_FP64 && out.precision != DFPR_FP32_KAHAN) ||
        (out.mode != DFPR_SYNC && out.mode != DFPR_ASYNC) ||
        (out.loop != DFPR_LOOP_LAUNCHES && out.loop != DFPR_LOOP_DEVICE))
        return set_error(DFPR_E_ARG, "invalid parameters");
    return DFPR_OK;
}

IterArgs iter_args(dfpr_graph *g, const dfpr_params &p, uint32_t sbase)
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
    a.ctl = g->ctl;
    a.mirror = g->ctl_host;
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
    // In the asynchronous form too: a copy taken when a workgroup starts
    // holds values the one rank vector had during this launch, which an
    // in-place sweep may read (on R-MAT scale 22 the same iterations and
    // error against the reference, 5% less time)
    a.hub = kHubRows;
    return a;
}

// Take a stamp base for a new call; stamps of earlier calls are all below it.
static int take_base(dfpr_graph *g, int32_t max_iters, uint32_t *base)
{
    const uint64_t span = (uint64_t)max_iters + 2;
    if ((uint64_t)g->next_base + span >= 0xF0000000ull) {
        int rc = launch_fill_u32(g, g->stamp, (uint64_t)g->n, 0);
        if (!rc) rc = launch_fill_u32(g, g->xstamp, (uint64_t)g->n, 0);
        if (!rc && g->mstamp) rc = launch_fill_u32(g, g->mstamp, (uint64_t)g->n, 0);
        if (!rc && g->mxstamp) rc = launch_fill_u32(g, g->mxstamp, (uint64_t)g->n, 0);
        if (rc) return rc;
        g->next_base = 1;
        g->last_iters = -1;           // the last update's marks are gone
    }
    *base = g->next_base;
    g->next_base += (uint32_t)span;
    return DFPR_OK;
}

// Run iterations it0, it0+1, ... until the device sets the stop flag (or,
// in the FP32 phase, the phase-end flag).  The phase starts on buffer
// `base`; iteration i reads buffer base ^ ((i - it0) & 1), or, in the
// asynchronous form (FP64 only), reads and writes buffer `base` in place.
// *res_buf receives the buffer holding the result.  Iterations are enqueued in
// chunks, up to two at a time; when a chunk completes the host reads the
// control block it left and sizes the next chunk from the observed
// geometric decay of Delta R, less what is still queued, so few launches
// run after convergence and the device does not wait for the host.
// Workgroups for the next chunk of a call still on the class lists: what
// the current lists need, times four and plus 64 for the frontier to grow
// within the chunk, at least one per CU.  Any grid gives the same result
// (the work is grid-strided); a small frontier just skips empty workgroups.
static uint32_t sparse_grid(const dfpr_graph *g, const Ctl &c)
{
    uint64_t nwu = 0;
    for (int b = 0; b < kBins - 1; b++) {
        const uint64_t rows = kWave / group_of(b);
        nwu += (c.live[b] + rows - 1) / rows;
    }
    const uint64_t need = std::max<uint64_t>(c.live[kBins - 1], (nwu + kWavesPerBlock - 1) /
                                                                     kWavesPerBlock);
    const uint64_t lo = std::min<uint64_t>(256, (uint64_t)g->grid);
    return (uint32_t)std::min<uint64_t>(g->grid, std::max<uint64_t>(lo, need * 4 + 64));
}

// One launch of the small-frontier loop from iteration it0 on buffer
// `base`, on the graph's stream; the host reads its final state from
// g->ctl_host after the stream has passed evc[0].
static int launch_small_loop(dfpr_graph *g, IterArgs a, bool f32, int it0, int base, int slot)
{
    LoopArgs L{};
    for (int b = 0; b < 2; b++) {
        L.R[b] = g->R[b];
        L.C[b] = g->C[b];
        L.C32[b] = g->C32[b];
    }
    L.base = base;
    L.it0 = it0;
    L.it_start = it0;
    L.limit = kLoopRows;
    L.bar = slot;
    a.mirror = g->ctl_host;
    void *args[] = {&a, &L};
    const void *fn = f32 ? reinterpret_cast<const void *>(&k_loop<true>)
                         : reinterpret_cast<const void *>(&k_loop<false>);
    DFPR_HIP(hipLaunchCooperativeKernel(fn, dim3(kLoopGrid), dim3(kBlock), args, 0, g->stream));
    DFPR_HIP(hipEventRecord(g->evc[0], g->stream));
    return DFPR_OK;
}

static int run_loop(dfpr_graph *g, const dfpr_params &p, bool df, bool f32, uint32_t sbase,
                    int it0, int base, int *res_buf, int small_slot = -1)
{
    IterArgs a = iter_args(g, p, sbase);
    const bool async = p.mode == DFPR_ASYNC && !f32;
    // Up to two chunks are in flight: while the host waits for the older
    // one and reads the control block it left in its own mirror, the newer
    // one keeps the device busy.  Chunk c uses mirror, completion event and
    // profiling events of slot c & 1.
    Ctl *const mirror[2] = {g->ctl_host, g->ctl_host + 1};
    struct Chunk {
        int k, slot;
    };
    Chunk q[2];
    int nq = 0, next_it = it0, nchunks = 0, chunk = 4, fin = 0;
    // iterations to keep queued beyond the last state read; until a state
    // is known, two chunks of four
    int target = 8, cap = 4;
    bool stop = false;
    uint32_t gsz = (uint32_t)g->grid;
    // walks of the full schedule run a wide kernel: Static and Naive-dynamic
    // from the start, Dynamic Frontier once a state shows the full schedule
    bool wide = DFPR_WIDE && !df;
    double prev_dr = -1.0;
    int prev_it = it0;
    *res_buf = base;
    // Dynamic Frontier on the class lists, if asked for: the first
    // iterations, while the frontier is small, run inside one launch of the
    // small-frontier loop
    if (df && !async && small_slot >= 0 && g->coop && p.loop == DFPR_LOOP_DEVICE &&
        p.max_iters > it0) {
        DFPR_CHECK_RC(launch_small_loop(g, a, f32, it0, base, small_slot));
        DFPR_HIP(hipEventSynchronize(g->evc[0]));
        const Ctl &st = *g->ctl_host;
        if (st.loop_fail) return set_error(DFPR_E_DEVICE, "small-frontier loop: grid barrier timed out");
        next_it = std::max(it0, (int)st.iterations);
        g->loop_iters += next_it - it0;
        // its work is not part of the iteration kernel's profile
        g->prof_base[0] = (int64_t)st.verts;
        g->prof_base[1] = (int64_t)st.edges;
        g->prof_base[2] = (int64_t)st.xverts;
        g->prof_base[3] = (int64_t)st.xedges;
        g->prof_base[4] = (int64_t)st.marked;
        if (st.done || (f32 && st.phase_end)) stop = true;
        else if (!st.dense) gsz = sparse_grid(g, st);
    }
    auto launch = [&](int k) -> int {
        const int slot = nchunks & 1;
        a.mirror = mirror[slot];
        hipEvent_t *ev = g->evk + slot * 2 * kLoopChunk;
        for (int j = 0; j < k; j++) {
            const int i = next_it + j;
            const int src = async ? base : base ^ ((i - it0) & 1);
            const int dst = async ? base : src ^ 1;
            a.Rc = g->R[src];
            a.Cc = g->C[src];
            a.Rn = g->R[dst];
            a.Cn = g->C[dst];
            a.C32c = g->C32[src];
            a.C32n = g->C32[src ^ 1];
            a.it = i;
            if (g->prof.enabled) DFPR_HIP(hipEventRecord(ev[2 * j], g->stream));
            if (wide) {
                IterArgs aw = a;
                if (!df) {
                    aw.hub = a.hub ? kWideHub : 0u;
                    k_iter_wide<false, false, kWideWaves, kWideHub>
                        <<<g->grid_wide, kWideWaves * kWave, 0, g->stream>>>(aw);
                } else if (f32) {
                    // FP32 contributions: the same LDS holds twice the entries
                    aw.hub = a.hub ? kWideDfHub * DFPR_WIDE_F32_MUL : 0u;
                    k_iter_wide<true, true, kWideDfWaves, kWideDfHub>
                        <<<g->grid_wide_df, kWideDfWaves * kWave, 0, g->stream>>>(aw);
                } else {
                    aw.hub = a.hub ? kWideDfHub : 0u;
                    k_iter_wide<true, false, kWideDfWaves, kWideDfHub>
                        <<<g->grid_wide_df, kWideDfWaves * kWave, 0, g->stream>>>(aw);
                }
            }
            else if (!df) k_iter<false, false><<<gsz, kBlock, 0, g->stream>>>(a);
            else if (f32) k_iter<true, true><<<gsz, kBlock, 0, g->stream>>>(a);
            else k_iter<true, false><<<gsz, kBlock, 0, g->stream>>>(a);
            if (g->prof.enabled) DFPR_HIP(hipEventRecord(ev[2 * j + 1], g->stream));
            k_final<<<1, kFinalThreads, 0, g->stream>>>(a, df ? 1 : 0, f32 ? 1 : 0,
                                                         j == k - 1 ? 1 : 0);
        }
        DFPR_HIP(hipGetLastError());
        DFPR_HIP(hipEventRecord(g->evc[slot], g->stream));
        q[nq++] = Chunk{k, slot};
        next_it += k;
        nchunks++;
        return DFPR_OK;
    };
    while (true) {
        int queued = 0;
        for (int t = 0; t < nq; t++) queued += q[t].k;
        while (!stop && nq < 2 && queued < target && next_it < p.max_iters) {
            const int k = std::min(std::min(target - queued, cap), p.max_iters - next_it);
            const int rc = launch(k);
            if (rc) return rc;
            queued += k;
        }
        if (nq == 0) break;
        const Chunk c = q[0];
        q[0] = q[1];
        nq--;
        // the chunk's last k_final, or the one that ended the call or the
        // phase, left the control block in the chunk's mirror
        DFPR_HIP(hipEventSynchronize(g->evc[c.slot]));
        if (g->prof.enabled) {
            // the iteration kernel alone, launch by launch
            const hipEvent_t *ev = g->evk + c.slot * 2 * kLoopChunk;
            for (int j = 0; j < c.k; j++) {
                float ms = 0.f;
                DFPR_HIP(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
                g->prof.ms += ms;
            }
            g->prof.launches += c.k;
        }
        if (stop) continue;             // later chunks return at once
        const Ctl &st = *mirror[c.slot];
        if (st.done || (f32 && st.phase_end)) {
            stop = true;
            fin = c.slot;
            continue;
        }
        // iterations still needed after this state, from the observed
        // geometric decay of Delta R
        gsz = df && !st.dense ? sparse_grid(g, st) : (uint32_t)g->grid;
        wide = DFPR_WIDE && (!df || st.dense);
        const double dr = st.final_linf;
        const int its = st.iterations;
        int need = std::min(chunk * 2, 32);
        // the FP32 phase ends at the larger of tol and its resolution
        // floor (see final_body); the FP64 loop at tol
        const double goal = f32 ? std::max(p.tol, st.final_rmax * 0x1p-22) : p.tol;
        if (prev_dr > 0.0 && dr > 0.0 && dr < prev_dr && its > prev_it && goal > 0.0) {
            const double rate = std::pow(dr / prev_dr, 1.0 / (its - prev_it));
            const double left = std::ceil(std::log(goal / dr) / std::log(rate));
            if (std::isfinite(left)) need = (int)std::min<double>(kLoopChunk, std::max(1.0, left));
        }
        prev_dr = dr;
        prev_it = its;
        chunk = need;
        cap = kLoopChunk;
        // at least one more iteration if nothing is queued: the call is not over
        target = std::max(need, nq > 0 ? 0 : 1);
    }
    if (fin == 1) *mirror[0] = *mirror[1];   // the final state goes to the main mirror
    if (p.max_iters <= it0) {
        DFPR_CHECK_RC(ctl_to_host(g));
        DFPR_HIP(hipStreamSynchronize(g->stream));
    }
    const Ctl &c = *g->ctl_host;
    *res_buf = async ? base : base ^ ((c.iterations - it0) & 1);
    if (g->prof.enabled) {
        const int64_t dv = (int64_t)c.verts - g->prof_base[0];
        const int64_t de = (int64_t)c.edges - g->prof_base[1];
        const int64_t dxv = (int64_t)c.xverts - g->prof_base[2];
        const int64_t dxe = (int64_t)c.xedges - g->prof_base[3];
        const int64_t dmk = (int64_t)c.marked - g->prof_base[4];
        g->prof.rows += dv;
        g->prof.edges += de;
        g->prof.exp_rows += dxv;
        g->prof.exp_edges += dxe;
        g->prof.marked += dmk;
        // per processed row: worklist entry 4 B, row start and length 8 B,
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
        g->prof_base[4] = (int64_t)c.marked;
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
    st->loop_iterations = g->loop_iters;
    st->frontier_tol_used = df ? c.ftol_used : 0.0;
    st->final_linf = c.final_linf;
    float ms = 0.f, ms0 = 0.f, ms1 = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev0, g->ev1);
    (void)hipEventElapsedTime(&ms0, g->ev0, g->ev_mid);
    (void)hipEventElapsedTime(&ms1, g->ev_mid, g->ev1);
    st->ms_device = ms;
    st->ms_mark = ms0;
    st->ms_iter = ms1;
    st->ms_apply = g->last_apply_ms;
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
        rc = ranks_from_caller(g, prev, prev_dev, g->R[cur]);
        if (rc) return rc;
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[cur], g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    } else if (!use_resident) {
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, nullptr, g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    }
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters, g->sparse_limit, 1, g->ctl_host, p.tol,
                           p.frontier_tol);
    DFPR_HIP(hipGetLastError());
    int res = cur;
    g->refine_sweeps = 0;
    g->loop_iters = 0;
    std::memset(g->prof_base, 0, sizeof(g->prof_base));
    DFPR_HIP(hipEventRecord(g->ev_mid, s));
    rc = run_loop(g, p, false, false, 0, 0, cur, &res);
    if (rc) return rc;
    k_copy2<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[res], g->R[res ^ 1], g->C[res],
                                             g->C[res ^ 1]);
    g->cur = res;
    DFPR_HIP(hipEventRecord(g->ev1, s));
    if (ranks_out) {
        rc = ranks_to_caller(g, g->R[res], ranks_out, out_dev);
        if (rc) return rc;
    }
    DFPR_HIP(hipStreamSynchronize(s));
    fill_stats(g, st, false);
    return DFPR_OK;
}

// Everything of a Dynamic Frontier call before its iterations, enqueued on
// the graph's stream: optional previous ranks, a stamp base, the initial
// marking of the batch (device arrays) and the snapshot of iteration 0.
// Returns the stamp base.
int df_begin(dfpr_graph *g, const dfpr_params &p, int64_t nd, const int32_t *bds,
             const int32_t *bdd, int64_t ni, const int32_t *bis, const int32_t *bid,
             const double *prev, int prev_dev, uint32_t *sbase_out, int32_t *lists)
{
    if (!lists) lists = g->ap.batch_dev + 2 * (nd + ni);
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    const int cur = g->cur;
    int rc = DFPR_OK;
    if (prev) {
        rc = ranks_from_caller(g, prev, prev_dev, g->R[cur]);
        if (rc) return rc;
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[cur], g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    }
    uint32_t sbase = 0;
    rc = take_base(g, p.max_iters, &sbase);
    if (rc) return rc;
    // the initial marking decides on the device whether the batch's
    // sources reach enough vertices to start on the full schedule
    const int dense = 0;
    IterArgs a = iter_args(g, p, sbase);
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (nd + ni > 0) {
        k_validate<<<blocks_for(nd + ni), kBlock, 0, s>>>(n, nd, bds, bdd, ni, bis, bid, g->ctl);
        launch_initial_marking(g, a, nd, bds, bdd, ni, bis, dense, lists);
    }
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters, g->sparse_limit, dense, g->ctl_host, p.tol,
                           p.frontier_tol);
    if (p.precision == DFPR_FP32_KAHAN)
        k_c32_init<<<blocks_for(n), kBlock, 0, s>>>(n, g->C[cur], g->C32[0], g->C32[1]);
    DFPR_HIP(hipGetLastError());
    g->refine_sweeps = 0;
    g->loop_iters = 0;
    std::memset(g->prof_base, 0, sizeof(g->prof_base));
    *sbase_out = sbase;
    return DFPR_OK;
}

// End of the FP32 phase (precision form).  If the call is over (the cap),
// rebuild the FP64 contributions from the ranks; otherwise renormalise the
// ranks to sum 1 in FP64 and rebuild the FP64 contributions, so FP64
// iterations can continue over the same marks from buffer `res`.
int df_phase_end(dfpr_graph *g, int res, bool call_done)
{
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    if (call_done) {
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[res], g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    } else {
        k_sum_part<<<kSumBlocks, kBlock, 0, s>>>(n, g->R[res], g->scratch_sum);
        k_sum_final<<<1, kBlock, 0, s>>>(g->scratch_sum, kSumBlocks, g->ctl);
        k_renorm<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[res], g->R[res ^ 1], g->C[0], g->C[1],
                                                  g->csr[1].cnt, g->ctl);
    }
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

// After the last iteration (result in buffer `res`): bring the other buffer
// up to date on the processed rows, count the marks, and make the result
// the resident ranks.
int df_finish(dfpr_graph *g, uint32_t sbase, int res, int32_t iters)
{
    const int32_t n = g->n;
    k_finish<<<std::min(blocks_for(n), 2048), kBlock, 0, g->stream>>>(
        n, g->stamp, sbase, sbase + (uint32_t)iters, g->R[res], g->R[res ^ 1], g->C[res],
        g->C[res ^ 1], g->ctl, g->bins, g->n);
    DFPR_HIP(hipGetLastError());
    g->cur = res;
    g->last_base = sbase;
    g->last_iters = iters;
    return DFPR_OK;
}

// A Dynamic Frontier call.  `staging` (device arrays only): a caller-chosen
// buffer of 4 (nd + ni) ints for the staged batch and the marking's source
// lists, in place of the library's own; such a call allocates nothing.
static int df_impl(dfpr_graph *g, const dfpr_params *pp, int64_t nd, const int32_t *ds,
                   const int32_t *dd, int64_t ni, const int32_t *is, const int32_t *id,
                   int on_device, const double *prev, double *ranks_out, dfpr_stats *st,
                   int32_t *staging = nullptr)
{
    dfpr_params p;
    int rc = check_params(pp, p);
    if (rc) return rc;
    if (staging && !on_device) return set_error(DFPR_E_ARG, "staging needs device arrays");
    if (nd < 0 || ni < 0 || (nd && (!ds || !dd)) || (ni && (!is || !id)))
        return set_error(DFPR_E_ARG, "bad batch arrays");
    if (!on_device) {
        rc = check_ids_host(g->n, nd, ds, dd);
        if (!rc) rc = check_ids_host(g->n, ni, is, id);
        if (rc) return rc;
    }
    BusyGuard guard(g);
    if (!guard.ok) return set_error(DFPR_E_BUSY, "graph in use");
    hipStream_t s = g->stream;
    DFPR_HIP(hipEventRecord(g->ev0, s));
    const int32_t *bds, *bdd, *bis, *bid;
    if (staging) rc = stage_batch_into(g, nd, ds, dd, ni, is, id, staging, &bds, &bdd, &bis, &bid);
    else rc = stage_batch(g, nd, ds, dd, ni, is, id, on_device, &bds, &bdd, &bis, &bid);
    if (rc) return rc;
    const int cur = g->cur;
    uint32_t sbase = 0;
    rc = df_begin(g, p, nd, bds, bdd, ni, bis, bid, prev, on_device, &sbase,
                  staging ? staging + 2 * (nd + ni) : nullptr);
    if (rc) return rc;
    DFPR_HIP(hipEventRecord(g->ev_mid, s));
    int res = cur;
    if (p.precision == DFPR_FP32_KAHAN) {
        // FP32 phase on FP32 copies of the contributions
        rc = run_loop(g, p, true, true, sbase, 0, cur, &res, 0);
        if (rc) return rc;
        if (g->ctl_host->err)
            return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
        const bool done = g->ctl_host->done != 0;
        rc = df_phase_end(g, res, done);
        if (rc) return rc;
        if (!done) {
            const int it0 = g->ctl_host->iterations;
            rc = run_loop(g, p, true, false, sbase, it0, res, &res, 1);
            if (rc) return rc;
            g->refine_sweeps = g->ctl_host->iterations - it0;
        }
    } else {
        rc = run_loop(g, p, true, false, sbase, 0, cur, &res, 0);
        if (rc) return rc;
    }
    const int32_t iters = g->ctl_host->iterations;
    if (g->ctl_host->err) return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
    rc = df_finish(g, sbase, res, iters);
    if (rc) return rc;
    DFPR_HIP(hipEventRecord(g->ev1, s));
    if (ranks_out) {
        rc = ranks_to_caller(g, g->R[res], ranks_out, on_device);
        if (rc) return rc;
    }
    DFPR_CHECK_RC(ctl_to_host(g));
    DFPR_HIP(hipStreamSynchronize(s));
    fill_stats(g, st, true);
    return DFPR_OK;
}

int df_device_staged(dfpr_graph *g, const dfpr_params *pp, int64_t nd, const int32_t *ds,
                     const int32_t *dd, int64_t ni, const int32_t *is, const int32_t *id,
                     const double *prev, double *ranks_out, dfpr_stats *st, int32_t *staging)
{
    return df_impl(g, pp, nd, ds, dd, ni, is, id, 1, prev, ranks_out, st, staging);
}

// Workgroups for a traversal level of `q` light vertices (a wave per 64),
// with room for the queue to grow sixteenfold within a chunk of levels; a
// level with heavy vertices gets the whole grid.
static uint32_t bfs_grid(const dfpr_graph *g, uint64_t q, uint64_t heavy)
{
    if (heavy) return (uint32_t)g->grid;
    const uint64_t blocks = (q + (uint64_t)kBlock - 1) / kBlock;
    return (uint32_t)std::min<uint64_t>(g->grid, std::max<uint64_t>(256, blocks * 16));
}

static BfsQueues bfs_queues(dfpr_graph *g, int64_t L)
{
    const size_t n = (size_t)g->n;
    int32_t *light = g->bfs_q, *heavy = g->bfs_q + 3 * n;
    uint32_t *qn = g->ctl->qn, *qhn = g->ctl->qhn;   // device addresses
    const int r0 = (int)(L % 3), r1 = (int)((L + 1) % 3), r2 = (int)((L + 2) % 3);
    BfsQueues q;
    q.in = light + r0 * n;
    q.hin = heavy + r0 * n;
    q.nin = qn + r0;
    q.nhin = qhn + r0;
    q.out = light + r1 * n;
    q.hout = heavy + r1 * n;
    q.nout = qn + r1;
    q.nhout = qhn + r1;
    q.clear = qn + r2;
    q.hclear = qhn + r2;
    return q;
}

// The traversal on the graph's stream: seed with the batch sources and
// deletion targets, then levels in chunks between host looks, until a
// level queues nothing.  Reached vertices end with stamp a.sbase.
static int traverse(dfpr_graph *g, const IterArgs &a, int64_t nd, const int32_t *bds,
                    const int32_t *bdd, int64_t ni, const int32_t *bis, bool append)
{
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    if (!g->bfs_q) DFPR_HIP(hipMalloc(&g->bfs_q, (size_t)6 * n * sizeof(int32_t)));
    // the seed fills the queues that level 0 reads: those of a level -1
    // (which reads and clears nothing)
    BfsQueues q0 = bfs_queues(g, 2);
    k_bfs_seed<<<std::min(blocks_for(nd + ni), 2048), kBlock, 0, s>>>(a, nd, bds, bdd, ni, bis,
                                                                   q0, append ? 1 : 0);
    DFPR_HIP(hipGetLastError());
    uint32_t grid = (uint32_t)g->grid;
    int chunk = 1;
    for (int64_t L = 0; L <= (int64_t)n;) {
        for (int j = 0; j < chunk; j++, L++)
            k_bfs_level<<<grid, kBlock, 0, s>>>(a, bfs_queues(g, L), append ? 1 : 0);
        DFPR_HIP(hipGetLastError());
        DFPR_CHECK_RC(ctl_to_host(g));
        DFPR_HIP(hipStreamSynchronize(s));
        const Ctl &c = *g->ctl_host;
        const uint32_t next = c.qn[L % 3], nexth = c.qhn[L % 3];
        if (c.err || (next == 0 && nexth == 0)) break;
        grid = bfs_grid(g, next, nexth);
        chunk = std::min(chunk * 2, 16);
    }
    return DFPR_OK;
}

// Dynamic Traversal PageRank (Section 3.3.2): the reachable set is marked
// before the first iteration and never grows, so the iterations are those
// of Dynamic Frontier with no expansion.  Always FP64.
static int dt_impl(dfpr_graph *g, const dfpr_params *pp, int64_t nd, const int32_t *ds,
                   const int32_t *dd, int64_t ni, const int32_t *is, const int32_t *id,
                   int on_device, const double *prev, double *ranks_out, dfpr_stats *st)
{
    dfpr_params p;
    int rc = check_params(pp, p);
    if (rc) return rc;
    p.precision = DFPR_FP64;
    p.frontier_tol = INFINITY;   // no vertex joins during the iterations
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
    const int32_t *bds, *bdd, *bis, *bid;
    rc = stage_batch(g, nd, ds, dd, ni, is, id, on_device, &bds, &bdd, &bis, &bid);
    if (rc) return rc;
    const int cur = g->cur;
    if (prev) {
        rc = ranks_from_caller(g, prev, on_device, g->R[cur]);
        if (rc) return rc;
        k_init_ranks<<<blocks_for(n), kBlock, 0, s>>>(n, g->R[cur], g->R[0], g->R[1], g->C[0],
                                                      g->C[1], g->csr[1].cnt);
    }
    uint32_t sbase = 0;
    rc = take_base(g, p.max_iters, &sbase);
    if (rc) return rc;
    IterArgs a = iter_args(g, p, sbase);
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (nd + ni > 0) {
        k_validate<<<blocks_for(nd + ni), kBlock, 0, s>>>(n, nd, bds, bdd, ni, bis, bid, g->ctl);
        rc = traverse(g, a, nd, bds, bdd, ni, bis, false);
        if (rc) return rc;
    }
    // the reachable set is usually most of the graph: the iterations walk
    // the full schedule and read the stamps, no class lists are built
    k_snap<<<1, 1, 0, s>>>(g->ctl, p.max_iters, g->sparse_limit, 1, g->ctl_host, p.tol,
                           p.frontier_tol);
    DFPR_HIP(hipGetLastError());
    g->refine_sweeps = 0;
    g->loop_iters = 0;
    std::memset(g->prof_base, 0, sizeof(g->prof_base));
    DFPR_HIP(hipEventRecord(g->ev_mid, s));
    int res = cur;
    rc = run_loop(g, p, true, false, sbase, 0, cur, &res);
    if (rc) return rc;
    const int32_t iters = g->ctl_host->iterations;
    if (g->ctl_host->err) return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
    rc = df_finish(g, sbase, res, iters);
    if (rc) return rc;
    DFPR_HIP(hipEventRecord(g->ev1, s));
    if (ranks_out) {
        rc = ranks_to_caller(g, g->R[res], ranks_out, on_device);
        if (rc) return rc;
    }
    DFPR_CHECK_RC(ctl_to_host(g));
    DFPR_HIP(hipStreamSynchronize(s));
    fill_stats(g, st, true);
    return DFPR_OK;
}

// Stamp arrays of the marking-only calls (dfpr_mark_affected,
// dfpr_mark_reachable), allocated on first use.  Keeping them apart from
// the iterations' stamps leaves the marks of the last update readable.
static int marking_stamps(dfpr_graph *g)
{
    if (g->mstamp) return DFPR_OK;
    const size_t bytes = (size_t)g->n * sizeof(uint32_t);
    DFPR_HIP(hipMalloc(&g->mstamp, bytes));
    hipError_t e = hipMalloc(&g->mxstamp, bytes);
    if (e != hipSuccess) {
        (void)hipFree(g->mstamp);
        g->mstamp = nullptr;
        return hip_fail(e, "hipMalloc(marking stamps)");
    }
    DFPR_CHECK_RC(launch_fill_u32(g, g->mstamp, (uint64_t)g->n, 0));
    DFPR_CHECK_RC(launch_fill_u32(g, g->mxstamp, (uint64_t)g->n, 0));
    return DFPR_OK;
}

}  // namespace dfpr

using namespace dfpr;

extern "C" {

int dfpr_set_ranks(dfpr_graph *g, const double *ranks, int on_device)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    BusyGuard guard(g);
    if (!guard.ok) return set_error(DFPR_E_BUSY, "graph in use");
    const int32_t n = g->n;
    hipStream_t s = g->stream;
    if (ranks) {
        const int rc = ranks_from_caller(g, ranks, on_device, g->R[0]);
        if (rc) return rc;
    }
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

int dfpr_pagerank_dynamic_traversal(dfpr_graph *g, const dfpr_params *p, int64_t n_del,
                                    const int32_t *del_src, const int32_t *del_dst,
                                    int64_t n_ins, const int32_t *ins_src,
                                    const int32_t *ins_dst, const double *prev,
                                    double *ranks_out, dfpr_stats *st)
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    return dt_impl(g, p, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 0, prev, ranks_out, st);
}

int dfpr_mark_reachable(dfpr_graph *g, int64_t n_del, const int32_t *del_src,
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
    rc = stage_batch(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 0, &bds, &bdd, &bis,
                     &bid);
    dfpr_params p;
    dfpr_params_default(&p);
    uint32_t sbase = 0;
    if (!rc) rc = marking_stamps(g);
    if (!rc) rc = take_base(g, 0, &sbase);
    if (rc) return rc;
    IterArgs a = iter_args(g, p, sbase);
    a.stamp = g->mstamp;
    a.xstamp = g->mxstamp;
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    DFPR_HIP(hipGetLastError());
    if (n_del + n_ins > 0) {
        rc = traverse(g, a, n_del, bds, bdd, n_ins, bis, false);
        if (rc) return rc;
    }
    std::vector<uint32_t> st(n);
    DFPR_HIP(hipMemcpyAsync(st.data(), g->mstamp, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    for (int32_t v = 0; v < n; v++) flags_out[v] = st[g->ext2int_h[v]] == sbase ? 1 : 0;
    return DFPR_OK;
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
    rc = stage_batch(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 0, &bds, &bdd, &bis,
                     &bid);
    dfpr_params p;
    dfpr_params_default(&p);
    uint32_t sbase = 0;
    if (!rc) rc = marking_stamps(g);
    if (!rc) rc = take_base(g, 0, &sbase);
    if (rc) return rc;
    IterArgs a = iter_args(g, p, sbase);
    a.stamp = g->mstamp;
    a.xstamp = g->mxstamp;
    k_reset<<<1, 1, 0, s>>>(g->ctl);
    if (n_del + n_ins > 0)
        launch_initial_marking(g, a, n_del, bds, bdd, n_ins, bis, 1,
                               g->ap.batch_dev + 2 * (n_del + n_ins));
    DFPR_HIP(hipGetLastError());
    std::vector<uint32_t> st(n);
    DFPR_HIP(hipMemcpyAsync(st.data(), g->mstamp, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    for (int32_t v = 0; v < n; v++) flags_out[v] = st[g->ext2int_h[v]] == sbase ? 1 : 0;
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
    for (int32_t v = 0; v < n; v++) {
        const uint32_t x = st[g->ext2int_h[v]];
        flags_out[v] = (g->last_iters >= 0 && x >= lo && x <= hi) ? 1 : 0;
    }
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
