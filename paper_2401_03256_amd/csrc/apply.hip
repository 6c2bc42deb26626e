// Device batch applier: E <- (E minus deletions) union insertions on both
// CSRs (Section 3.2; self-loops are permanent, Section 5.1.4).
//
// Steps, all on the device:
//   1. keys: each batch entry becomes, per orientation, the 64-bit key
//      row << 33 | col << 1 | type (type 0 = deletion, 1 = insertion);
//      self-loop deletions become a sentinel that sorts last; an id outside
//      [0, n) sets the error flag and every later step does nothing.
//   2. sort: each workgroup sorts a tile of 2048 keys in LDS (bitonic), then
//      merge passes double the sorted runs (each key finds its output slot by
//      a binary search in the other run).
//   3. heads: the first key of each row opens a "touched row" entry; rows
//      whose capacity fits in LDS go to one list, larger rows to another.
//   4. merge: one workgroup per touched row.  It copies the row (LDS or a
//      global slab), works out which deletions hit a present edge and which
//      insertions add a new one, and writes every surviving entry and every
//      new entry straight to its final slot (positions from prefix counts
//      and binary searches), keeping the row sorted.  The out-orientation
//      pass also refreshes the row's contribution R/|out|.
//   5. a row whose slots are too few is written instead to fresh slots
//      taken from the free space at the end of the index array (one atomic
//      add on the array's top).  Only when that space is used up is the row
//      left for a re-layout: new capacities, a prefix sum, a copy of every
//      row to its new place with fresh free space, and the merge is run
//      again from the round that did not fit.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"

namespace dfpr {

#ifndef DFPR_SORT_TILE
#define DFPR_SORT_TILE 512
#endif
constexpr int kTile = DFPR_SORT_TILE;   // keys sorted per tile in LDS (a multiple of kBlock)
static_assert(kTile % kBlock == 0, "a tile is ranked by whole workgroups");
constexpr int kOpsLds = 1024;  // batch entries of one row per round
constexpr int kRowLds = 4096;  // rows up to this capacity are copied to LDS
#ifndef DFPR_BIG_GRID
#define DFPR_BIG_GRID 256
#endif
constexpr int kBigGrid = DFPR_BIG_GRID;   // workgroups (and slabs) per orientation for larger rows
// Workgroups of the three row kernels.  Each workgroup of the out-row pass
// leaves its applied counts in its own pair of slots of ApplyBufs::part,
// folded once afterwards: tens of thousands of atomics on one address
// would serialise.
constexpr int kCopyUnroll = 8;  // row entries loaded per thread before use
constexpr int kTinyGrid = 4096;
constexpr int kSmallGrid = 8192;
constexpr int kPartSlots = 2 * (kTinyGrid + kSmallGrid + kBigGrid);

__device__ inline uint32_t key_row(uint64_t k) { return (uint32_t)(k >> 33); }
__device__ inline int32_t key_col(uint64_t k) { return (int32_t)((k >> 1) & 0xFFFFFFFFull); }

template <typename T>
__device__ inline uint32_t lower_bound_dev(const T *a, uint32_t len, T x)
{
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename T>
__device__ inline uint32_t upper_bound_dev(const T *a, uint32_t len, T x)
{
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}


// First index at or after lo whose element is not below x, for a cursor that
// only moves forward (every element before lo is below x): steps that double
// from lo, then a binary search inside the last step.
template <typename T>
__device__ inline uint32_t gallop_dev(const T *a, uint32_t lo, uint32_t len, T x)
{
    uint32_t hi = lo, step = 1;
    while (hi < len && a[hi] < x) {
        lo = hi + 1;
        hi += step;
        step <<= 1;
    }
    if (hi > len) hi = len;
    return lo + lower_bound_dev(a + lo, hi - lo, x);
}

struct ApplyArgs {
    int32_t n;
    int64_t nd, ni;
    const int32_t *ds, *dd, *is, *id;
    uint64_t *keys[2];          // unsorted / sorted keys per orientation
    uint32_t *tiny_list[2], *small_list[2], *big_list[2], *ovf_list[2];
    int32_t *ovf_need[2];
    uint32_t *beg[2], *cnt[2], *cap[2];
    int32_t *idx[2];
    uint64_t slots[2];
    double *R0, *R1, *C0, *C1;
    int32_t *slab;
    uint64_t slab_stride;
    unsigned long long *part;   // null: add applied counts to Ctl directly
    Ctl *ctl;
};

// Applied counts of one out-row workgroup: into its slots of part, or
// straight into Ctl when there are no slots.  Thread 0 holds the sums.
__device__ inline void put_applied(const ApplyArgs &a, uint32_t slot, unsigned long long d,
                                   unsigned long long i)
{
    if (a.part) {
        a.part[2 * slot] = d;
        a.part[2 * slot + 1] = i;
    } else if (d | i) {
        atomicAdd(&a.ctl->applied[0], d);
        atomicAdd(&a.ctl->applied[1], i);
    }
}

// Sum the applied counts that the launched workgroups of the three row
// kernels left in part into Ctl.
constexpr int kFoldThreads = 1024;

__global__ __launch_bounds__(kFoldThreads) void k_apply_fold(const unsigned long long *part,
                                                       uint32_t tiny_grid, uint32_t small_grid,
                                                       Ctl *ctl)
{
    __shared__ unsigned long long s[2][kFoldThreads];
    const uint32_t base[3] = {0, kTinyGrid, kTinyGrid + kSmallGrid};
    const uint32_t used[3] = {tiny_grid, small_grid, kBigGrid};
    unsigned long long d = 0, i = 0;
    for (int r = 0; r < 3; r++)
        for (uint32_t k = base[r] + threadIdx.x; k < base[r] + used[r]; k += kFoldThreads) {
            d += part[2 * k];
            i += part[2 * k + 1];
        }
    s[0][threadIdx.x] = d;
    s[1][threadIdx.x] = i;
    __syncthreads();
    for (int st = kFoldThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s[0][threadIdx.x] += s[0][threadIdx.x + st];
            s[1][threadIdx.x] += s[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->applied[0] += s[0][0];
        ctl->applied[1] += s[1][0];
    }
}

__global__ void k_apply_reset(Ctl *ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->err = 0;
        for (int o = 0; o < 2; o++) {
            ctl->ntiny[o] = ctl->nsmall[o] = ctl->nbig[o] = ctl->novf[o] = 0;
            ctl->applied[o] = 0;
        }
    }
}

__global__ void k_apply_keys(ApplyArgs a)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.nd + a.ni) return;
    const bool del = i < a.nd;
    const int32_t s = del ? a.ds[i] : a.is[i - a.nd];
    const int32_t d = del ? a.dd[i] : a.id[i - a.nd];
    if (s < 0 || s >= a.n || d < 0 || d >= a.n) {
        atomicOr(&a.ctl->err, 1u);
        a.keys[0][i] = a.keys[1][i] = kSentinel;
        return;
    }
    if (del && s == d) {   // self-loops are never deleted
        a.keys[0][i] = a.keys[1][i] = kSentinel;
        return;
    }
    const uint64_t t = del ? 0 : 1;
    a.keys[0][i] = ((uint64_t)d << 33) | ((uint64_t)(uint32_t)s << 1) | t;   // in-CSR: row = dst
    a.keys[1][i] = ((uint64_t)s << 33) | ((uint64_t)(uint32_t)d << 1) | t;   // out-CSR: row = src
}

// Sort tiles of up to kTile keys, in -> out; grid.y = orientation.  Rank
// sort: workgroup (t, q) loads tile t into LDS and ranks keys
// q * kBlock .. q * kBlock + kBlock - 1 of it, one per thread, by counting the
// keys that order before it (equal keys by position, so the sort is
// stable); each key is stored at its rank.  No barriers inside the count,
// and kTile / kBlock workgroups share a tile.
__global__ __launch_bounds__(kBlock) void k_tile_sort(const uint64_t *in0, uint64_t *out0,
                                                      const uint64_t *in1, uint64_t *out1,
                                                      uint32_t len)
{
    constexpr uint32_t kParts = kTile / kBlock;
    constexpr int kStep = 8;
    __shared__ uint64_t s[kTile];
    const uint64_t *in = blockIdx.y ? in1 : in0;
    uint64_t *out = blockIdx.y ? out1 : out0;
    const uint32_t base = (blockIdx.x / kParts) * kTile;
    const uint32_t cnt = min((uint32_t)kTile, len - base);
    const uint32_t i = (blockIdx.x % kParts) * kBlock + threadIdx.x;
    if ((blockIdx.x % kParts) * kBlock >= cnt) return;      // uniform
    for (uint32_t k = threadIdx.x; k < cnt; k += kBlock) s[k] = in[base + k];
    __syncthreads();
    if (i >= cnt) return;
    const uint64_t mine = s[i];
    uint32_t rank = 0;
    uint32_t j0 = 0;
    for (; j0 + kStep <= cnt; j0 += kStep) {
        uint64_t y[kStep];
#pragma unroll
        for (int u = 0; u < kStep; u++) y[u] = s[j0 + u];
#pragma unroll
        for (int u = 0; u < kStep; u++)
            rank += (y[u] < mine || (y[u] == mine && j0 + u < i)) ? 1u : 0u;
    }
    for (uint32_t j = j0; j < cnt; j++) {
        const uint64_t y = s[j];
        rank += (y < mine || (y == mine && j < i)) ? 1u : 0u;
    }
    out[base + rank] = mine;
}

// Merge sorted runs of `width` keys pairwise: in -> out.
__global__ void k_merge_pass(const uint64_t *in0, uint64_t *out0, const uint64_t *in1,
                             uint64_t *out1, uint32_t len, uint32_t width)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const uint64_t *in = blockIdx.y ? in1 : in0;
    uint64_t *out = blockIdx.y ? out1 : out0;
    const uint64_t key = in[i];
    const uint32_t start = (i / (2 * width)) * (2 * width);
    const uint32_t mid = min(start + width, len), end = min(start + 2 * width, len);
    uint32_t pos;
    if (i < mid) pos = (i - start) + lower_bound_dev(in + mid, end - mid, key);
    else pos = (i - mid) + upper_bound_dev(in + start, mid - start, key);
    out[start + pos] = key;
}

// Open one touched-row entry at the first key of every row.
__global__ void k_heads(ApplyArgs a, uint32_t len)
{
    if (a.ctl->err) return;
    const int o = blockIdx.y;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t *keys = a.keys[o];
    // rows by the capacity they had before the batch and their number of
    // batch entries: 0 = at most kWave of each (one wave), 1 = copied to
    // LDS (one workgroup), 2 = larger (workgroup with a global slab)
    bool head = false;
    int which_row = 1;
    if (i < len) {
        const uint64_t k = keys[i];
        if (k != kSentinel) {
            const uint32_t r = key_row(k);
            head = i == 0 || key_row(keys[i - 1]) != r;
            if (head) {
                // a row can grow by its number of entries over the rounds
                // of the merge: only rows that stay within kRowLds go to LDS
                const uint64_t cap = a.cap[o][r];
                const uint32_t nops = gallop_dev(keys, i, len, (uint64_t)(r + 1) << 33) - i;
                if (cap + nops > (uint64_t)kRowLds) which_row = 2;
                else if (cap <= (uint64_t)kWave && nops <= (uint32_t)kWave) which_row = 0;
            }
        }
    }
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int which = 0; which < 3; which++) {
        const bool take = head && which_row == which;
        const unsigned long long m = __ballot(take);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        uint32_t *cnt = which == 0 ? &a.ctl->ntiny[o] : which == 1 ? &a.ctl->nsmall[o]
                                                                    : &a.ctl->nbig[o];
        uint32_t *list = which == 0 ? a.tiny_list[o] : which == 1 ? a.small_list[o]
                                                                   : a.big_list[o];
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
        base = __shfl(base, leader);
        if (take) list[base + __popcll(m & below)] = i;
    }
}

// Lanes 0 .. len-1 hold v in ascending order: how many of them are below x.
// Every lane of the wave calls it.
template <class T>
__device__ inline uint32_t lanes_below(T v, uint32_t len, T x)
{
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t step = kWave; step > 0; step >>= 1) {
        const T y = __shfl(v, (int)min(pos + step - 1, (uint32_t)kWave - 1));
        if (pos + step <= len && y < x) pos += step;
    }
    return pos;
}

__device__ inline unsigned long long lanes_mask(uint32_t k)
{
    return k >= (uint32_t)kWave ? ~0ull : (1ull << k) - 1ull;
}

// Rows of at most kWave slots touched by at most kWave batch entries: one
// wave per row, entries and operations one per lane, with the same rules as
// the workgroup path below (distinct operations; a deletion takes effect if
// the entry is present, an insertion if it is absent or deleted by the same
// batch; survivors shift left past effective deletions and right past
// effective insertions; a row that outgrows its slots moves to free space at
// the top, or is left for a re-layout).
__global__ __launch_bounds__(kBlock) void k_apply_tiny(ApplyArgs a, uint32_t len)
{
    const int o = blockIdx.y;
    Ctl *ctl = a.ctl;
    if (ctl->err) return;
    const uint32_t count = ctl->ntiny[o];
    const uint64_t *keys = a.keys[o];
    uint32_t *beg_a = a.beg[o], *cnt_a = a.cnt[o], *cap_a = a.cap[o];
    int32_t *idx = a.idx[o];
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t waves = gridDim.x * kWavesPerBlock;
    unsigned long long sum_del = 0, sum_ins = 0;
    for (uint32_t t = wave; t < count; t += waves) {
        const uint32_t start = a.tiny_list[o][t];
        // operations (sorted by column, deletion before insertion)
        const uint64_t kl = (uint32_t)lane < len - start ? keys[start + lane] : kSentinel;
        const uint32_t row = key_row(__shfl(kl, 0));
        const bool isop = kl != kSentinel && key_row(kl) == row;
        const uint32_t nops = (uint32_t)__popcll(__ballot(isop));
        const uint64_t k = isop ? kl : ~0ull;
        const uint32_t beg = beg_a[row], cap = cap_a[row], c = cnt_a[row];
        const uint64_t kp = __shfl_up(k, 1);
        const bool first = isop && (lane == 0 || kp != k);
        const int32_t col = isop ? key_col(k) : INT32_MAX;
        const bool del = first && !(k & 1), ins = first && (k & 1);
        // the row's entries (ascending)
        const int32_t e = (uint32_t)lane < c ? idx[beg + lane] : INT32_MAX;
        const uint32_t pb = lanes_below(e, c, col);
        const int32_t at = __shfl(e, (int)min(pb, (uint32_t)kWave - 1));
        const bool present = isop && pb < c && at == col;
        const bool deleted_too = lane > 0 && isop && key_col(kp) == col && !(kp & 1);
        const unsigned long long mdel = __ballot(del && present);
        const unsigned long long mins = __ballot(ins && (!present || deleted_too));
        const uint32_t ndel = (uint32_t)__popcll(mdel), nins = (uint32_t)__popcll(mins);
        const uint32_t nc = c - ndel + nins;
        uint32_t dest = beg, ncap = cap;
        int ok = 1;
        if (lane == 0 && nc > cap) {
            const uint64_t want = (uint64_t)nc + (nc / 8 > 2 ? nc / 8 : 2);
            const uint64_t top = atomicAdd(&ctl->top[o], (unsigned long long)want);
            if (want <= 0xFFFFFFFFull && top + want <= a.slots[o]) {
                dest = (uint32_t)top;
                ncap = (uint32_t)want;
                atomicMax(&ctl->max_cap[o], (uint32_t)want);
            } else {
                ok = 0;
                const uint32_t slot = atomicAdd(&ctl->novf[o], 1u);
                a.ovf_list[o][slot] = start;
                a.ovf_need[o][slot] = (int32_t)(c + nops);
            }
        }
        dest = __shfl(dest, 0);
        ncap = __shfl(ncap, 0);
        ok = __shfl(ok, 0);
        if (!ok) continue;
        // entry e: operations below it, and whether a deletion removes it
        const uint32_t ob = lanes_below(col, nops, e);
        const int32_t ocol = __shfl(col, (int)min(ob, (uint32_t)kWave - 1));
        const bool gone = ob < nops && ((mdel >> ob) & 1ull) && ocol == e;
        if ((uint32_t)lane < c && !gone)
            idx[dest + lane - __popcll(mdel & lanes_mask(ob)) + __popcll(mins & lanes_mask(ob))] =
                e;
        // insertion: entries below it that survive, then earlier insertions
        const uint32_t lo = lanes_below(col, nops, col);
        if ((mins >> lane) & 1ull)
            idx[dest + pb - __popcll(mdel & lanes_mask(lo)) + __popcll(mins & below)] = col;
        if (lane == 0) {
            cnt_a[row] = nc;
            beg_a[row] = dest;
            cap_a[row] = ncap;
            if (o == 1) {
                sum_del += ndel;
                sum_ins += nins;
                // |out(row)| changed: refresh the stored contributions
                a.C0[row] = a.R0[row] / (double)nc;
                a.C1[row] = a.R1[row] / (double)nc;
            }
        }
    }
    if (o == 1) {
        __shared__ unsigned long long s_sum[2][kWavesPerBlock];
        const int w = threadIdx.x / kWave;
        if (lane == 0) {
            s_sum[0][w] = sum_del;
            s_sum[1][w] = sum_ins;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 1; k < kWavesPerBlock; k++) {
                sum_del += s_sum[0][k];
                sum_ins += s_sum[1][k];
            }
            put_applied(a, blockIdx.x, sum_del, sum_ins);
        }
    }
}

// Exclusive prefix sum of in[0 .. len) (len <= 4 * kBlock) into out[0 .. len],
// out[len] = total.  All threads of the workgroup call it.
__device__ inline void block_scan_u8(const uint8_t *in, uint32_t len, uint32_t *out, uint32_t *tmp)
{
    if (len <= (uint32_t)kWave) {
        // one wave: a ballot holds every flag
        if (threadIdx.x < kWave) {
            const uint32_t lane = threadIdx.x;
            const unsigned long long m = __ballot(lane < len && in[lane] != 0);
            if (lane < len) out[lane] = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) out[len] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        return;
    }
    const uint32_t t = threadIdx.x, b = t * 4;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        v[r] = b + r < len ? in[b + r] : 0;
        sum += v[r];
    }
    tmp[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kBlock; off <<= 1) {
        uint32_t x = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += x;
        __syncthreads();
    }
    uint32_t ex = tmp[t] - sum;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        if (b + r < len) out[b + r] = ex;
        ex += v[r];
    }
    if (t == kBlock - 1) out[len] = tmp[t];
    __syncthreads();
}

// Position of the first entry of a sorted row in global memory (c entries)
// not below x, given smp[k] = row[k * stride] for k < ns = ceil(c / stride):
// a search in the samples leaves fewer than stride candidates, halved while
// more than kCopyUnroll remain, then counted with independent loads.
__device__ inline uint32_t sampled_lower_bound(const int32_t *row, uint32_t c, const int32_t *smp,
                                               uint32_t ns, uint32_t stride, int32_t x)
{
    const uint32_t k = lower_bound_dev(smp, ns, x);
    if (k == 0) return 0;
    uint32_t lo = (k - 1) * stride + 1;  // row[lo - 1] < x
    uint32_t hi = min(k * stride, c);    // hi == c or row[hi] >= x
    while (hi - lo > (uint32_t)kCopyUnroll) {
        const uint32_t mid = (lo + hi) >> 1;
        if (row[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    uint32_t below = 0;
#pragma unroll
    for (int u = 0; u < kCopyUnroll; u++)
        if (lo + u < hi) below += row[lo + u] < x;
    return lo + below;
}

// Merge the batch entries of touched rows into their rows.  Rows up to
// kRowLds entries are copied to LDS.  Larger rows (BIG) are searched through
// LDS samples; a row that moves to fresh slots is read in place, and a row
// that stays copies only the part from its first operation on to a global
// slab, since the entries before it keep their slots.
template <bool BIG>
__global__ __launch_bounds__(kBlock) void k_apply_rows(ApplyArgs a, uint32_t len, int only_o)
{
    __shared__ int32_t s_d[kOpsLds];
    __shared__ int32_t s_i[kOpsLds];
    __shared__ uint8_t s_fd[kOpsLds];
    __shared__ uint8_t s_fi[kOpsLds];
    __shared__ uint32_t s_pd[kOpsLds + 1];
    __shared__ uint32_t s_pi[kOpsLds + 1];
    __shared__ uint32_t s_ipos[kOpsLds];  // row position of each insertion
    __shared__ uint32_t s_tmp[kBlock];
    __shared__ int32_t s_row[kRowLds];    // the row, or (BIG) its samples
    __shared__ uint32_t s_dest, s_ncap, s_first;
    __shared__ int s_ok;

    const int o = only_o >= 0 ? only_o : blockIdx.y;
    if (only_o >= 0 && blockIdx.y > 0) return;
    Ctl *ctl = a.ctl;
    if (ctl->err) return;
    const uint32_t count = BIG ? ctl->nbig[o] : ctl->nsmall[o];
    const uint32_t *list = BIG ? a.big_list[o] : a.small_list[o];
    const uint64_t *keys = a.keys[o];
    uint32_t *beg_a = a.beg[o], *cnt_a = a.cnt[o], *cap_a = a.cap[o];
    int32_t *idx = a.idx[o];
    // one slab per (workgroup, orientation): both orientations run at once
    int32_t *slab = BIG ? a.slab + ((uint64_t)blockIdx.y * kBigGrid + blockIdx.x) * a.slab_stride
                        : nullptr;

    unsigned long long sum_del = 0, sum_ins = 0;  // thread 0, out-rows
    for (uint32_t t = blockIdx.x; t < count; t += gridDim.x) {
        // list entries point at the first batch key of the row, or, for a
        // re-run after a re-layout, at the first key of the round that did
        // not fit (earlier rounds were applied)
        const uint32_t start = list[t];
        const uint32_t row = key_row(keys[start]);
        const uint32_t end = gallop_dev(keys, start, len, (uint64_t)(row + 1) << 33);
        for (uint32_t j0 = start; j0 < end; j0 += kOpsLds) {
            const uint32_t beg = beg_a[row], cap = cap_a[row];
            const uint32_t nops = min((uint32_t)kOpsLds, end - j0);
            // distinct deletions / insertions of this round (keys are sorted
            // by col then type, so repeats are adjacent)
            for (uint32_t q = threadIdx.x; q < nops; q += kBlock) {
                const uint32_t j = j0 + q;
                const uint64_t k = keys[j];
                const bool first = j == 0 || keys[j - 1] != k;
                s_fd[q] = first && !(k & 1);
                s_fi[q] = first && (k & 1);
            }
            __syncthreads();
            block_scan_u8(s_fd, nops, s_pd, s_tmp);
            block_scan_u8(s_fi, nops, s_pi, s_tmp);
            for (uint32_t q = threadIdx.x; q < nops; q += kBlock) {
                const int32_t col = key_col(keys[j0 + q]);
                if (s_fd[q]) s_d[s_pd[q]] = col;
                if (s_fi[q]) s_i[s_pi[q]] = col;
            }
            const uint32_t nd = s_pd[nops], ni = s_pi[nops];
            const uint32_t c = cnt_a[row];
            if (BIG && c > a.slab_stride) {
                // the slab cannot hold this row: leave it to a re-layout
                if (threadIdx.x == 0) {
                    const uint32_t slot = atomicAdd(&ctl->novf[o], 1u);
                    a.ovf_list[o][slot] = j0;
                    a.ovf_need[o][slot] = (int32_t)(c + (end - j0));
                }
                __syncthreads();
                break;
            }
            const int32_t *grow = idx + beg;  // the row in global memory
            // BIG: one sample every `stride` entries, at most kRowLds
            const uint32_t stride = BIG ? max(1u, (c + kRowLds - 1) / kRowLds) : 1;
            const uint32_t ns = BIG ? (c + stride - 1) / stride : c;
            // kCopyUnroll loads in flight per thread
            for (uint32_t k0 = threadIdx.x; k0 < ns; k0 += kBlock * kCopyUnroll) {
                int32_t v[kCopyUnroll];
#pragma unroll
                for (int u = 0; u < kCopyUnroll; u++) {
                    const uint32_t k = k0 + u * kBlock;
                    v[u] = k < ns ? grow[k * stride] : 0;
                }
#pragma unroll
                for (int u = 0; u < kCopyUnroll; u++) {
                    const uint32_t k = k0 + u * kBlock;
                    if (k < ns) s_row[k] = v[u];
                }
            }
            if (threadIdx.x == 0) s_first = c;
            __syncthreads();
            // which entries take effect; s_first: where the first operation
            // falls in the row
            for (uint32_t q = threadIdx.x; q < nd; q += kBlock) {
                const int32_t col = s_d[q];
                uint32_t pos;
                bool present;
                if (BIG) {
                    pos = sampled_lower_bound(grow, c, s_row, ns, stride, col);
                    present = pos < c && grow[pos] == col;
                } else {
                    pos = lower_bound_dev(s_row, c, col);
                    present = pos < c && s_row[pos] == col;
                }
                s_fd[q] = present;
                if (q == 0) atomicMin(&s_first, pos);
            }
            for (uint32_t q = threadIdx.x; q < ni; q += kBlock) {
                const int32_t col = s_i[q];
                uint32_t pos;
                bool present;
                if (BIG) {
                    pos = sampled_lower_bound(grow, c, s_row, ns, stride, col);
                    present = pos < c && grow[pos] == col;
                } else {
                    pos = lower_bound_dev(s_row, c, col);
                    present = pos < c && s_row[pos] == col;
                }
                const uint32_t pd = lower_bound_dev(s_d, nd, col);
                const bool deleted = pd < nd && s_d[pd] == col;
                s_fi[q] = !present || deleted;
                s_ipos[q] = pos;
                if (q == 0) atomicMin(&s_first, pos);
            }
            __syncthreads();
            block_scan_u8(s_fd, nd, s_pd, s_tmp);
            block_scan_u8(s_fi, ni, s_pi, s_tmp);
            const uint32_t ndel = s_pd[nd], nins = s_pi[ni];
            const uint32_t nc = c - ndel + nins;
            if (threadIdx.x == 0) {
                s_dest = beg;
                s_ncap = cap;
                s_ok = 1;
                if (nc > cap) {
                    // move the row to fresh slots at the top of the array
                    const uint64_t want = (uint64_t)nc + (nc / 8 > 2 ? nc / 8 : 2);
                    const uint64_t at = atomicAdd(&ctl->top[o], (unsigned long long)want);
                    if (want <= 0xFFFFFFFFull && at + want <= a.slots[o]) {
                        s_dest = (uint32_t)at;
                        s_ncap = (uint32_t)want;
                        atomicMax(&ctl->max_cap[o], (uint32_t)want);
                    } else {
                        s_ok = 0;
                        const uint32_t slot = atomicAdd(&ctl->novf[o], 1u);
                        a.ovf_list[o][slot] = j0;
                        a.ovf_need[o][slot] = (int32_t)(c + (end - j0));
                    }
                }
            }
            __syncthreads();
            if (!s_ok) break;
            const uint32_t dest = s_dest;
            // Entries [lo, c) are rewritten: all of them when the row moves,
            // else (BIG) those from the first operation on, staged in the
            // slab so that no slot is written before it is read.
            const bool moved = dest != beg;
            const uint32_t lo = BIG && !moved ? s_first : 0;
            if (BIG && !moved) {
                for (uint32_t p0 = lo + threadIdx.x; p0 < c; p0 += kBlock * kCopyUnroll) {
                    int32_t v[kCopyUnroll];
#pragma unroll
                    for (int u = 0; u < kCopyUnroll; u++) {
                        const uint32_t p = p0 + u * kBlock;
                        v[u] = p < c ? grow[p] : 0;
                    }
#pragma unroll
                    for (int u = 0; u < kCopyUnroll; u++) {
                        const uint32_t p = p0 + u * kBlock;
                        if (p < c) slab[p - lo] = v[u];
                    }
                }
                __syncthreads();
            }
            // surviving entries shift left past deletions, right past
            // insertions; a thread's entries ascend, so its cursors into the
            // sorted operations only move forward
            uint32_t kd = 0, ki = 0;
            for (uint32_t p0 = lo + threadIdx.x; p0 < c; p0 += kBlock * kCopyUnroll) {
                int32_t v[kCopyUnroll];
#pragma unroll
                for (int u = 0; u < kCopyUnroll; u++) {
                    const uint32_t p = p0 + u * kBlock;
                    v[u] = p >= c ? 0 : !BIG ? s_row[p] : moved ? grow[p] : slab[p - lo];
                }
#pragma unroll
                for (int u = 0; u < kCopyUnroll; u++) {
                    const uint32_t p = p0 + u * kBlock;
                    if (p >= c) break;
                    const int32_t e = v[u];
                    kd = gallop_dev(s_d, kd, nd, e);
                    if (kd < nd && s_d[kd] == e) continue;
                    ki = gallop_dev(s_i, ki, ni, e);
                    idx[dest + p - s_pd[kd] + s_pi[ki]] = e;
                }
            }
            for (uint32_t q = threadIdx.x; q < ni; q += kBlock) {
                if (!s_fi[q]) continue;
                const int32_t col = s_i[q];
                const uint32_t below = s_ipos[q] - s_pd[lower_bound_dev(s_d, nd, col)];
                idx[dest + s_pi[q] + below] = col;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                cnt_a[row] = nc;
                beg_a[row] = dest;
                cap_a[row] = s_ncap;
                if (o == 1) {
                    sum_del += ndel;
                    sum_ins += nins;
                    // |out(row)| changed: refresh the stored contributions
                    a.C0[row] = a.R0[row] / (double)nc;
                    a.C1[row] = a.R1[row] / (double)nc;
                }
            }
            __syncthreads();
        }
    }
    if (o == 1 && threadIdx.x == 0)
        put_applied(a, (BIG ? kTinyGrid + kSmallGrid : kTinyGrid) + blockIdx.x, sum_del, sum_ins);
}

// ---- re-layout of one orientation after slack overflow --------------------

__global__ void k_caps(int32_t n, const uint32_t *cap, uint64_t *caps)
{
    for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += gridDim.x * blockDim.x)
        caps[r] = r < n ? (uint64_t)cap[r] : 0;
}

// Grown capacity for each row left for the re-layout (in both tables).
__global__ void k_ovf_caps(uint32_t count, const uint32_t *list, const int32_t *need,
                           const uint64_t *keys, uint64_t *caps, uint32_t *cap)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t d = (uint64_t)need[i];
    const uint32_t r = key_row(keys[list[i]]);
    const uint64_t c = d + (d / 8 > 2 ? d / 8 : 2);
    caps[r] = c;
    cap[r] = (uint32_t)c;
}

// exclusive scan of caps[0 .. len) in place, 3 phases, 2048 per workgroup
constexpr int kScanTile = 2048;

__global__ __launch_bounds__(kBlock) void k_scan_sums(const uint64_t *x, uint64_t len,
                                                      uint64_t *sums)
{
    __shared__ uint64_t s[kBlock];
    const uint64_t base = blockIdx.x * (uint64_t)kScanTile;
    uint64_t acc = 0;
    for (int r = 0; r < kScanTile / kBlock; r++) {
        uint64_t i = base + threadIdx.x * (kScanTile / kBlock) + r;
        if (i < len) acc += x[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kBlock) void k_scan_top(uint64_t *sums, uint32_t nb)
{
    __shared__ uint64_t s[kBlock];
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kBlock) {
        const uint32_t i = b0 + threadIdx.x;
        const uint64_t v = i < nb ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            uint64_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
        const uint64_t tot = s[kBlock - 1];
        __syncthreads();
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(uint64_t *x, uint64_t len,
                                                       const uint64_t *sums)
{
    __shared__ uint64_t s[kBlock];
    constexpr int per = kScanTile / kBlock;
    const uint64_t base = blockIdx.x * (uint64_t)kScanTile + threadIdx.x * per;
    uint64_t v[per], acc = 0;
    for (int r = 0; r < per; r++) {
        v[r] = base + r < len ? x[base + r] : 0;
        acc += v[r];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        uint64_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    uint64_t ex = sums[blockIdx.x] + s[threadIdx.x] - acc;
    for (int r = 0; r < per; r++) {
        if (base + r < len) x[base + r] = ex;
        ex += v[r];
    }
}

// copy every row's live entries to its new place (one wave per row)
__global__ __launch_bounds__(kBlock) void k_move_rows(int32_t n, uint32_t *beg,
                                                      const uint32_t *cnt, const int32_t *idx,
                                                      const uint64_t *nbeg, int32_t *nidx)
{
    const int lane = __lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave; r < n; r += waves) {
        const uint32_t b = beg[r], c = cnt[r];
        const uint64_t nb = nbeg[r];
        for (uint32_t k = lane; k < c; k += kWave) nidx[nb + k] = idx[b + k];
        if (lane == 0) beg[r] = (uint32_t)nb;
    }
}

static int ensure_apply_bufs(dfpr_graph *g, uint64_t B)
{
    ApplyBufs &ap = g->ap;
    if (B <= ap.cap) return DFPR_OK;
    const uint64_t cap = std::max<uint64_t>(B, 4096);
    for (int o = 0; o < 2; o++) {
        for (int k = 0; k < 2; k++) {
            (void)hipFree(ap.keys[o][k]);
            ap.keys[o][k] = nullptr;
            DFPR_HIP(hipMalloc(&ap.keys[o][k], cap * 8));
        }
        uint32_t **lists[4] = {&ap.tiny_list[o], &ap.small_list[o], &ap.big_list[o],
                               &ap.ovf_list[o]};
        for (auto l : lists) {
            (void)hipFree(*l);
            *l = nullptr;
            DFPR_HIP(hipMalloc(l, cap * 4));
        }
        (void)hipFree(ap.ovf_need[o]);
        ap.ovf_need[o] = nullptr;
        DFPR_HIP(hipMalloc(&ap.ovf_need[o], cap * 4));
    }
    if (!ap.part) DFPR_HIP(hipMalloc(&ap.part, (size_t)kPartSlots * 8));
    ap.cap = cap;
    return DFPR_OK;
}

// Bytes of the row slabs the applier keeps for a graph's current largest row.
int64_t apply_slab_bytes(const dfpr_graph *g)
{
    const uint64_t stride = std::max(g->csr[0].max_cap, g->csr[1].max_cap);
    return (int64_t)(stride * kBigGrid * 2 * 4);
}

static int ensure_slab(dfpr_graph *g)
{
    const uint64_t stride = std::max(g->csr[0].max_cap, g->csr[1].max_cap);
    const uint64_t need = stride * kBigGrid * 2;
    if (need <= g->ap.slab_ints && g->ap.slab) {
        g->ap.slab_stride = g->ap.slab_ints / (kBigGrid * 2);
        return DFPR_OK;
    }
    (void)hipFree(g->ap.slab);
    g->ap.slab = nullptr;
    DFPR_HIP(hipMalloc(&g->ap.slab, std::max<uint64_t>(need, 1) * 4));
    g->ap.slab_ints = need;
    g->ap.slab_stride = stride;
    return DFPR_OK;
}

static inline unsigned grid_for(uint64_t items, unsigned per = kBlock)
{
    return (unsigned)std::max<uint64_t>(1, (items + per - 1) / per);
}

// Copy a batch (host or device arrays) into the graph's staging buffer in
// internal ids; ids outside [0, n) become -1 and are rejected later.  The
// buffer keeps 2 (n_del + n_ins) more entries after the batch for the
// initial marking.
int stage_batch(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                int64_t n_ins, const int32_t *is, const int32_t *id, int on_device,
                const int32_t **dds, const int32_t **ddd, const int32_t **dis,
                const int32_t **did)
{
    ApplyBufs &ap = g->ap;
    hipStream_t s = g->stream;
    // the batch, then room for the two source lists of the initial marking
    const uint64_t need = 4 * (uint64_t)(n_del + n_ins);
    const int64_t tot = 2 * (n_del + n_ins);
    // work still reading the staging buffers is finished before they are
    // replaced or refilled
    if (need > ap.batch_cap || !ap.batch_dev || (!on_device && tot > 0))
        DFPR_HIP(hipStreamSynchronize(s));
    if (need > ap.batch_cap || !ap.batch_dev) {
        (void)hipFree(ap.batch_dev);
        ap.batch_dev = nullptr;
        const uint64_t cap = std::max<uint64_t>(need, 8192);
        DFPR_HIP(hipMalloc(&ap.batch_dev, cap * 4));
        ap.batch_cap = cap;
    }
    int32_t *p = ap.batch_dev;
    int32_t *dst[4] = {p, p + n_del, p + 2 * n_del, p + 2 * n_del + n_ins};
    const int32_t *src[4] = {ds, dd, is, id};
    const int64_t len[4] = {n_del, n_del, n_ins, n_ins};
    if (!on_device && tot > 0) {
        // one copy through a pinned buffer, then the ids mapped in place
        if ((uint64_t)tot > ap.batch_host_cap || !ap.batch_host) {
            if (ap.batch_host) (void)hipHostFree(ap.batch_host);
            ap.batch_host = nullptr;
            ap.batch_host_cap = 0;
            const uint64_t cap = std::max<uint64_t>(tot, 8192);
            DFPR_HIP(hipHostMalloc((void **)&ap.batch_host, cap * 4, hipHostMallocDefault));
            ap.batch_host_cap = cap;
        }
        int64_t at = 0;
        for (int k = 0; k < 4; k++) {
            if (len[k]) std::memcpy(ap.batch_host + at, src[k], (size_t)len[k] * 4);
            at += len[k];
        }
        DFPR_HIP(hipMemcpyAsync(p, ap.batch_host, (size_t)tot * 4, hipMemcpyHostToDevice, s));
        const int rc = map_ids(g, p, p, tot);
        if (rc) return rc;
    } else if (tot > 0) {
        const int rc = map_ids4(g, src, len, p);
        if (rc) return rc;
    }
    *dds = dst[0];
    *ddd = dst[1];
    *dis = dst[2];
    *did = dst[3];
    return DFPR_OK;
}

int stage_batch_into(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                     int64_t n_ins, const int32_t *is, const int32_t *id, int32_t *buf,
                     const int32_t **dds, const int32_t **ddd, const int32_t **dis,
                     const int32_t **did)
{
    const int32_t *src[4] = {ds, dd, is, id};
    const int64_t len[4] = {n_del, n_del, n_ins, n_ins};
    if (n_del + n_ins > 0) DFPR_CHECK_RC(map_ids4(g, src, len, buf));
    *dds = buf;
    *ddd = buf + n_del;
    *dis = buf + 2 * n_del;
    *did = buf + 2 * n_del + n_ins;
    return DFPR_OK;
}

static ApplyArgs apply_args(dfpr_graph *g)
{
    ApplyArgs a{};
    a.n = g->n;
    for (int o = 0; o < 2; o++) {
        a.tiny_list[o] = g->ap.tiny_list[o];
        a.small_list[o] = g->ap.small_list[o];
        a.big_list[o] = g->ap.big_list[o];
        a.ovf_list[o] = g->ap.ovf_list[o];
        a.ovf_need[o] = g->ap.ovf_need[o];
        a.beg[o] = g->csr[o].beg;
        a.cnt[o] = g->csr[o].cnt;
        a.cap[o] = g->csr[o].cap;
        a.idx[o] = g->csr[o].idx;
        a.slots[o] = g->csr[o].slots;
    }
    a.R0 = g->R[0];
    a.R1 = g->R[1];
    a.C0 = g->C[0];
    a.C1 = g->C[1];
    a.slab = g->ap.slab;
    a.slab_stride = g->ap.slab_stride;
    a.ctl = g->ctl;
    return a;
}

// Grow the rows of orientation o listed in the overflow list and move every
// row to a freshly laid out index array (with new free space at its end).
static int relayout(dfpr_graph *g, int o, uint32_t novf, const uint64_t *sorted_keys)
{
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    Csr &c = g->csr[o];
    // temporaries freed on every return (hipFree waits for the device)
    struct Tmp {
        uint64_t *p = nullptr;
        ~Tmp() { (void)hipFree(p); }
    } caps_buf, sums_buf;
    const uint64_t len = (uint64_t)n + 1;
    const uint32_t nb = (uint32_t)((len + kScanTile - 1) / kScanTile);
    DFPR_HIP(hipMalloc(&caps_buf.p, len * 8));
    DFPR_HIP(hipMalloc(&sums_buf.p, (uint64_t)nb * 8));
    uint64_t *const caps = caps_buf.p, *const sums = sums_buf.p;
    k_caps<<<grid_for(len), kBlock, 0, s>>>(n, c.cap, caps);
    k_ovf_caps<<<grid_for(novf), kBlock, 0, s>>>(novf, g->ap.ovf_list[o], g->ap.ovf_need[o],
                                                 sorted_keys, caps, c.cap);
    std::vector<int32_t> need(novf);
    DFPR_HIP(hipMemcpyAsync(need.data(), g->ap.ovf_need[o], (size_t)novf * 4,
                            hipMemcpyDeviceToHost, s));
    k_scan_sums<<<nb, kBlock, 0, s>>>(caps, len, sums);
    k_scan_top<<<1, kBlock, 0, s>>>(sums, nb);
    k_scan_apply<<<nb, kBlock, 0, s>>>(caps, len, sums);
    uint64_t packed = 0;
    DFPR_HIP(hipMemcpyAsync(&packed, caps + n, 8, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    const uint64_t slots = packed + std::max<uint64_t>(packed / 16, 1 << 16);
    if (slots > 0xFFFFFFFFull) return set_error(DFPR_E_LIMIT, "graph needs more than 2^32-1 edge slots");
    int32_t *nidx = nullptr;
    DFPR_HIP(hipMalloc(&nidx, slots * 4));
    k_move_rows<<<4096, kBlock, 0, s>>>(n, c.beg, c.cnt, c.idx, caps, nidx);
    DFPR_HIP(hipGetLastError());
    const unsigned long long top = packed;
    DFPR_HIP(hipMemcpyAsync(&g->ctl->top[o], &top, 8, hipMemcpyHostToDevice, s));
    DFPR_HIP(hipStreamSynchronize(s));
    (void)hipFree(c.idx);
    c.idx = nidx;
    c.slots = slots;
    for (int32_t d : need) {
        const uint64_t cap = (uint64_t)d + std::max<uint64_t>(2, (uint64_t)d / 8);
        c.max_cap = std::max<uint32_t>(c.max_cap, (uint32_t)cap);
    }
    return DFPR_OK;
}

int apply_batch_impl(dfpr_graph *g, int64_t n_del, const int32_t *ds, const int32_t *dd,
                     int64_t n_ins, const int32_t *is, const int32_t *id, int on_device,
                     int64_t applied[2])
{
    if (n_del < 0 || n_ins < 0 || (n_del && (!ds || !dd)) || (n_ins && (!is || !id)))
        return set_error(DFPR_E_ARG, "bad batch arrays");
    if (n_del + n_ins >= (1ll << 31)) return set_error(DFPR_E_ARG, "batch too large");
    if (!on_device) {
        int rc = check_ids_host(g->n, n_del, ds, dd);
        if (!rc) rc = check_ids_host(g->n, n_ins, is, id);
        if (rc) return rc;
    }
    if (applied) applied[0] = applied[1] = 0;
    g->last_apply_ms = 0.f;
    const uint32_t B = (uint32_t)(n_del + n_ins);
    if (B == 0) return DFPR_OK;
    int rc = ensure_apply_bufs(g, B);
    if (!rc) rc = ensure_slab(g);
    if (rc) return rc;
    hipStream_t s = g->stream;
    DFPR_HIP(hipEventRecord(g->ev_a0, s));
    rc = stage_batch(g, n_del, ds, dd, n_ins, is, id, on_device, &ds, &dd, &is, &id);
    if (rc) return rc;
    ApplyArgs a = apply_args(g);
    a.nd = n_del;
    a.ni = n_ins;
    a.ds = ds;
    a.dd = dd;
    a.is = is;
    a.id = id;
    a.keys[0] = g->ap.keys[0][0];
    a.keys[1] = g->ap.keys[1][0];
    k_apply_reset<<<1, 1, 0, s>>>(g->ctl);
    k_apply_keys<<<grid_for(B), kBlock, 0, s>>>(a);
    const unsigned tiles = (B + kTile - 1) / kTile;
    k_tile_sort<<<dim3(tiles * (kTile / kBlock), 2), kBlock, 0, s>>>(
        g->ap.keys[0][0], g->ap.keys[0][1], g->ap.keys[1][0], g->ap.keys[1][1], B);
    int pp = 1;
    for (uint32_t w = kTile; w < B; w *= 2) {
        k_merge_pass<<<dim3(grid_for(B), 2), kBlock, 0, s>>>(
            g->ap.keys[0][pp], g->ap.keys[0][pp ^ 1], g->ap.keys[1][pp], g->ap.keys[1][pp ^ 1], B,
            w);
        pp ^= 1;
    }
    a.keys[0] = g->ap.keys[0][pp];
    a.keys[1] = g->ap.keys[1][pp];
    k_heads<<<dim3(grid_for(B), 2), kBlock, 0, s>>>(a, B);
    // every workgroup writes its slots of part, so they need no clearing;
    // the fold reads the slots of the workgroups launched
    a.part = g->ap.part;
    const unsigned tiny_grid = std::min<unsigned>(grid_for(B, kWavesPerBlock), kTinyGrid);
    const unsigned small_grid = std::min<unsigned>(B, kSmallGrid);
    k_apply_tiny<<<dim3(tiny_grid, 2), kBlock, 0, s>>>(a, B);
    k_apply_rows<false><<<dim3(small_grid, 2), kBlock, 0, s>>>(a, B, -1);
    k_apply_rows<true><<<dim3(kBigGrid, 2), kBlock, 0, s>>>(a, B, -1);
    k_apply_fold<<<1, kFoldThreads, 0, s>>>(a.part, tiny_grid, small_grid, a.ctl);
    DFPR_HIP(hipGetLastError());
    DFPR_HIP(hipEventRecord(g->ev_a1, s));
    DFPR_CHECK_RC(ctl_to_host(g));
    DFPR_HIP(hipStreamSynchronize(s));
    if (g->ctl_host->err) return set_error(DFPR_E_RANGE, "vertex id outside [0, n) in the batch");
    for (int o = 0; o < 2; o++)
        g->csr[o].max_cap = std::max(g->csr[o].max_cap, g->ctl_host->max_cap[o]);
    for (int o = 0; o < 2; o++) {
        const uint32_t novf = g->ctl_host->novf[o];
        if (!novf) continue;
        rc = relayout(g, o, novf, a.keys[o]);
        if (!rc) rc = ensure_slab(g);
        if (rc) return rc;
        // run the merge again for the grown rows only, as "big" rows
        ApplyArgs b = apply_args(g);
        b.nd = a.nd;
        b.ni = a.ni;
        b.keys[0] = a.keys[0];
        b.keys[1] = a.keys[1];
        DFPR_HIP(hipMemcpyAsync(g->ap.big_list[o], g->ap.ovf_list[o], (size_t)novf * 4,
                                hipMemcpyDeviceToDevice, s));
        DFPR_HIP(hipMemcpyAsync(&g->ctl->nbig[o], &g->ctl->novf[o], 4, hipMemcpyDeviceToDevice, s));
        k_apply_rows<true><<<dim3(kBigGrid, 1), kBlock, 0, s>>>(b, B, o);
        DFPR_HIP(hipGetLastError());
        DFPR_HIP(hipEventRecord(g->ev_a1, s));
        DFPR_CHECK_RC(ctl_to_host(g));
        DFPR_HIP(hipStreamSynchronize(s));
        if (g->ctl_host->novf[o] != novf)
            return set_error(DFPR_E_DEVICE, "row still overflows after re-layout");
    }
    const int64_t eff_del = (int64_t)g->ctl_host->applied[0];
    const int64_t eff_ins = (int64_t)g->ctl_host->applied[1];
    g->m += eff_ins - eff_del;
    {
        float ms = 0.f;
        DFPR_HIP(hipEventElapsedTime(&ms, g->ev_a0, g->ev_a1));
        g->last_apply_ms = ms;
    }
    if (applied) {
        applied[0] = eff_del;
        applied[1] = eff_ins;
    }
    return DFPR_OK;
}

}  // namespace dfpr

using namespace dfpr;

extern "C" {

int dfpr_apply_batch(dfpr_graph *g, int64_t n_del, const int32_t *del_src, const int32_t *del_dst,
                     int64_t n_ins, const int32_t *ins_src, const int32_t *ins_dst,
                     int64_t applied[2])
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    if (__atomic_exchange_n(&g->busy, 1, __ATOMIC_ACQ_REL)) return set_error(DFPR_E_BUSY, "graph in use");
    int rc = apply_batch_impl(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 0, applied);
    __atomic_store_n(&g->busy, 0, __ATOMIC_RELEASE);
    return rc;
}

int dfpr_apply_batch_device(dfpr_graph *g, int64_t n_del, const int32_t *del_src,
                            const int32_t *del_dst, int64_t n_ins, const int32_t *ins_src,
                            const int32_t *ins_dst, int64_t applied[2])
{
    if (!g) return set_error(DFPR_E_ARG, "graph is NULL");
    if (__atomic_exchange_n(&g->busy, 1, __ATOMIC_ACQ_REL)) return set_error(DFPR_E_BUSY, "graph in use");
    int rc = apply_batch_impl(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, 1, applied);
    __atomic_store_n(&g->busy, 0, __ATOMIC_RELEASE);
    return rc;
}

}  // extern "C"
