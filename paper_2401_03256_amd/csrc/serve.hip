// Serving form: continuous batching of Dynamic Frontier updates over many
// resident graphs.
//
// Graphs stay resident on the device with their ranks.  Update requests
// (graph, batch, arrival time) wait in arrival order and are admitted into
// one of a few slots when (a) a slot is free, (b) their graph has no update
// in flight (one writer per graph, Section 3.2) and (c) the HBM budget
// covers the resident graphs plus the scratch of every admitted request.
// Admission applies the batch to the graph and runs the initial marking on
// a stream of its own, while the iterations of the requests already
// admitted keep running.
//
// Requests run in two lanes, each on its own stream.  A large graph (at
// least kLargeEdges edges: an iteration over its full schedule fills the
// GPU) takes the large lane, which holds one request at a time, so large
// requests run one after another in arrival order and never queue behind
// small ones.  The large lane keeps a second chunk of steps queued behind
// the one running, so its request does not wait for the host between
// chunks.  All other requests share the small lane: every step runs one
// iteration of each of them in one launch, each slot owning a range of
// workgroups sized for its graph, so small updates progress beside a large
// one instead of waiting for it.  While a large request runs, a small-lane
// step takes at most kSmallLaneBlocks workgroups.  FP64 slots and slots in
// the FP32 phase of the precision form share a launch.  Chunk lengths
// follow the observed geometric decay of Delta R of the slots (so a slot is
// retired soon after it converges); small-lane chunks are kept short while
// requests wait for a slot, because requests join and leave at chunk
// boundaries.  The host serves whichever lane finishes a chunk first.
//
// Each slot runs exactly the per-row code of the single-graph engine
// (iter.h) with the same class of every row, so a request's result does not
// depend on what else is in flight or on its lane.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "common.h"
#include "iter.h"
#include "serve_policy.h"

namespace dfpr {

constexpr int kMaxSlots = 8;
constexpr int kMaxChunk = 32;
constexpr int64_t kRequestBytesPerEntry = 96;   // device scratch per batch entry
constexpr double kChunkMsWhileWaiting = 1.0;   // chunk length while requests wait
constexpr int64_t kLargeEdges = int64_t(1) << 25;   // edges that put a graph in the large lane
constexpr int kLanes = 2;                      // 0: large graphs, one at a time; 1: the rest
constexpr int kDepth = 2;                      // chunks a lane may have in flight
// Workgroups of one small-lane step while a large request runs (0: no cap).
#ifndef DFPR_SMALL_LANE_BLOCKS
#define DFPR_SMALL_LANE_BLOCKS 512
#endif
constexpr uint32_t kSmallLaneBlocks = DFPR_SMALL_LANE_BLOCKS;

struct MultiArgs {
    int32_t nslots;
    uint32_t f32_mask;                 // slot s is in an FP32 phase
    uint32_t off[kMaxSlots + 1];       // slot s owns workgroups off[s] .. off[s+1]-1
    IterArgs s[kMaxSlots];
};
static_assert(sizeof(MultiArgs) <= 4096, "kernel arguments must fit in 4 KiB");

struct CtlGather {
    int32_t n;
    const Ctl *src[kMaxSlots];
    Ctl *dst;
};
static_assert(sizeof(Ctl) % 4 == 0, "control blocks are copied as words");

__global__ __launch_bounds__(kBlock, DFPR_ITER_WAVES_PER_SIMD) void k_iter_multi(MultiArgs m)
{
    __shared__ IterShared sh;
#if DFPR_HUB
    __shared__ double hub[kHubRows];
#else
    double *hub = nullptr;
#endif
    const uint32_t b = blockIdx.x;
    int s = 0;
    while (s + 1 < m.nslots && b >= m.off[s + 1]) s++;
    const uint32_t G = m.off[s + 1] - m.off[s];
    if ((m.f32_mask >> s) & 1u) iter_body<true, true>(m.s[s], b - m.off[s], G, sh, hub);
    else iter_body<true, false>(m.s[s], b - m.off[s], G, sh, hub);
}

// One workgroup per slot.
__global__ __launch_bounds__(kFinalThreads) void k_final_multi(MultiArgs m)
{
    __shared__ FinalShared sh;
    const int s = blockIdx.x;
    const IterArgs &a = m.s[s];
    const bool f32 = (m.f32_mask >> s) & 1u;
    final_body(a, true, f32, sh, false);
}

// Copy the control blocks of the slots into one array for one host copy.
__global__ __launch_bounds__(kBlock) void k_gather_ctl(CtlGather g)
{
    constexpr int words = (int)(sizeof(Ctl) / 4);
    for (int i = threadIdx.x; i < g.n * words; i += kBlock) {
        const int s = i / words, w = i % words;
        reinterpret_cast<uint32_t *>(g.dst + s)[w] =
            reinterpret_cast<const uint32_t *>(g.src[s])[w];
    }
}

// Workgroups that can have work in any iteration of a graph: the count of
// the full schedule over its class id ranges, which bounds every frontier.
static uint32_t blocks_bound(const dfpr_graph *g, uint32_t grid)
{
    const uint32_t *c = g->cls;
    // the self-loop rows one per lane; class b the range [c[kBins-1-b], c[kBins-b])
    uint64_t nwu = ((uint64_t)(c[kBins + 1] - c[kBins]) + kWave - 1) / kWave;
    for (int b = 0; b < kBins - 1; b++) {
        const uint64_t rows = kWave / group_of(b);
        nwu += ((uint64_t)(c[kBins - b] - c[kBins - 1 - b]) + rows - 1) / rows;
    }
    const uint64_t nbu = c[1] - c[0];
    const uint64_t wblocks = (nwu + kWavesPerBlock - 1) / kWavesPerBlock;
    return (uint32_t)std::max<uint64_t>(1, std::max(std::min<uint64_t>(grid, nbu),
                                                    std::min<uint64_t>(grid, wblocks)));
}

using Clock = std::chrono::steady_clock;

struct Request {
    int32_t gid = 0;
    double arrival_ms = 0.0;
    std::vector<int32_t> ds, dd, is, id;
    int64_t charge = 0;
    int state = 0;            // 0 waiting, 1 running, 2 done
    dfpr_request_result res{};
};

struct Slot {
    int64_t req = -1;
    uint32_t sbase = 0;
    int phase32 = 0;          // in the FP32 phase of the precision form
    int it0 = 0;              // first iteration of the current phase
    int base = 0;             // buffer the current phase started on
    int it = 0;               // iterations done at the last look
    int itq = 0;              // first iteration not yet queued
    uint32_t epoch = 0;       // changes when the slot changes request or phase
    uint32_t blocks = 1;      // workgroups in a coalesced launch
    double prev_dr = -1.0;    // Delta R and iteration count at the last look
    int prev_it = 0;
    int pred = 4;             // predicted iterations left in the phase
};

struct GraphEntry {
    dfpr_graph *g = nullptr;
    dfpr_params p{};
    int64_t bytes = 0;
    int busy = 0;
    int lane = 1;
};

// Device bytes a graph holds (CSRs, rank and contribution buffers, stamps,
// id maps, class lists, FP32 contributions).
static int64_t graph_bytes(const dfpr_graph *g)
{
    const int64_t n = g->n;
    int64_t b = 0;
    for (int o = 0; o < 2; o++) b += (int64_t)g->csr[o].slots * 4 + 3 * n * 4;
    b += 5 * n * 8 + 2 * n * 4 + 2 * n * 4 + (int64_t)kBins * n * 4 + 2 * n * 4;
    return b + apply_slab_bytes(g);   // the applier's row copies of long rows
}

static double pct(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double k = (v.size() - 1) * q / 100.0;
    const size_t lo = (size_t)std::floor(k), hi = (size_t)std::ceil(k);
    return v[lo] + (v[hi] - v[lo]) * (k - lo);
}

}  // namespace dfpr

struct dfpr_server {
    int32_t max_slots = 1;
    int64_t large_edges = dfpr::kLargeEdges;   // graphs this large take the large lane
    int64_t budget = 0;
    int64_t resident = 0;
    std::vector<dfpr::GraphEntry> graphs;
    std::vector<dfpr::Request> reqs;
    hipStream_t stream[dfpr::kLanes] = {};   // per lane: iterations, phase ends, finishing
    hipStream_t astream = nullptr;           // admission: apply + initial marking
    // per lane and chunk in flight: its end, its gathered control blocks
    // (kMaxSlots) and their pinned host copy
    hipEvent_t done[dfpr::kLanes][dfpr::kDepth] = {};
    dfpr::Ctl *ctl_dev[dfpr::kLanes][dfpr::kDepth] = {};
    dfpr::Ctl *ctl_pin[dfpr::kLanes][dfpr::kDepth] = {};
};

using namespace dfpr;

namespace dfpr {

static double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Admit request r into slot sl on the admission stream: apply the batch,
// then begin the update; returns when both are done on the device.
static int admit(dfpr_server *srv, int64_t r, Slot &sl, double now_ms)
{
    Request &q = srv->reqs[r];
    GraphEntry &ge = srv->graphs[q.gid];
    dfpr_graph *g = ge.g;
    q.state = 1;
    q.res.admit_ms = now_ms;
    g->stream = srv->astream;
    int rc = DFPR_OK;
    do {
        int64_t applied[2] = {0, 0};
        const int64_t nd = (int64_t)q.ds.size(), ni = (int64_t)q.is.size();
        rc = apply_batch_impl(g, nd, q.ds.data(), q.dd.data(), ni, q.is.data(), q.id.data(), 0,
                              applied);
        if (rc) break;
        q.res.applied[0] = applied[0];
        q.res.applied[1] = applied[1];
        const int32_t *bds, *bdd, *bis, *bid;
        rc = stage_batch(g, nd, q.ds.data(), q.dd.data(), ni, q.is.data(), q.id.data(), 0, &bds,
                         &bdd, &bis, &bid);
        if (rc) break;
        uint32_t sbase = 0;
        rc = df_begin(g, ge.p, nd, bds, bdd, ni, bis, bid, nullptr, 0, &sbase);
        if (rc) break;
        if (hipStreamSynchronize(srv->astream) != hipSuccess) {
            rc = set_error(DFPR_E_DEVICE, "admission failed on the device");
            break;
        }
        sl = Slot();
        sl.req = r;
        sl.sbase = sbase;
        sl.phase32 = ge.p.precision == DFPR_FP32_KAHAN ? 1 : 0;
        sl.base = g->cur;
        sl.blocks = blocks_bound(g, (uint32_t)g->grid);
    } while (0);
    g->stream = srv->stream[ge.lane];
    return rc;
}

// Enqueue K coalesced steps of the slots in the chunk, from each slot's
// first unqueued iteration, then one copy of their control blocks to the
// host (buffer `buf` of the lane).  With `cap` > 0 the slots share at most
// about `cap` workgroups, in proportion to their bounds (each slot walks its
// rows grid-stride, so the workgroup count changes no result).
static int launch_chunk(dfpr_server *srv, int lane, int buf, std::vector<Slot *> &cs, int K,
                        uint32_t cap)
{
    hipStream_t stream = srv->stream[lane];
    MultiArgs m{};
    m.nslots = (int32_t)cs.size();
    uint64_t want = 0;
    for (const Slot *sl : cs) want += sl->blocks;
    uint32_t at = 0;
    for (int i = 0; i < m.nslots; i++) {
        m.off[i] = at;
        uint32_t nb = cs[i]->blocks;
        if (cap && want > cap) nb = (uint32_t)std::max<uint64_t>(1, (uint64_t)nb * cap / want);
        at += nb;
        if (cs[i]->phase32) m.f32_mask |= 1u << i;
    }
    m.off[m.nslots] = at;
    for (int j = 0; j < K; j++) {
        for (int i = 0; i < m.nslots; i++) {
            Slot &sl = *cs[i];
            const Request &q = srv->reqs[sl.req];
            GraphEntry &ge = srv->graphs[q.gid];
            dfpr_graph *g = ge.g;
            IterArgs a = iter_args(g, ge.p, sl.sbase);
            a.mirror = nullptr;       // the slots' blocks come back gathered
            const int it = sl.itq + j;
            const int src = sl.base ^ ((it - sl.it0) & 1);
            a.Rc = g->R[src];
            a.Cc = g->C[src];
            a.Rn = g->R[src ^ 1];
            a.Cn = g->C[src ^ 1];
            a.C32c = g->C32[src];
            a.C32n = g->C32[src ^ 1];
            a.it = it;
            m.s[i] = a;
        }
        k_iter_multi<<<at, kBlock, 0, stream>>>(m);
        k_final_multi<<<m.nslots, kFinalThreads, 0, stream>>>(m);
    }
    CtlGather cg{};
    cg.n = m.nslots;
    for (int i = 0; i < m.nslots; i++) cg.src[i] = srv->graphs[srv->reqs[cs[i]->req].gid].g->ctl;
    cg.dst = srv->ctl_dev[lane][buf];
    k_gather_ctl<<<1, kBlock, 0, stream>>>(cg);
    DFPR_HIP(hipGetLastError());
    DFPR_HIP(hipMemcpyAsync(srv->ctl_pin[lane][buf], srv->ctl_dev[lane][buf],
                            m.nslots * sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    DFPR_HIP(hipEventRecord(srv->done[lane][buf], stream));
    for (Slot *sl : cs) sl->itq += K;
    return DFPR_OK;
}

// Predicted iterations left in a slot's phase, from the geometric decay of
// Delta R between two looks.
static void predict(Slot &sl, const Ctl &c, double tol)
{
    const double dr = c.final_linf;
    const int its = c.iterations;
    int next = std::min(sl.pred * 2, kMaxChunk);
    if (sl.prev_dr > 0.0 && dr > 0.0 && dr < sl.prev_dr && its > sl.prev_it && tol > 0.0) {
        const double rate = std::pow(dr / sl.prev_dr, 1.0 / (its - sl.prev_it));
        const double need = std::ceil(std::log(tol / dr) / std::log(rate));
        if (std::isfinite(need)) next = (int)std::min<double>(kMaxChunk, std::max(1.0, need));
    }
    sl.prev_dr = dr;
    sl.prev_it = its;
    sl.pred = next;
}

// A chunk in flight: its slots (with their epochs at launch), its steps,
// the lane buffer its control blocks go to and its host launch time.
struct Chunk {
    std::vector<Slot *> cs;
    std::vector<uint32_t> epoch;
    int K = 0;
    int buf = 0;
    Clock::time_point t;
};

// A lane's chunks in flight, oldest first.  The large lane keeps a second
// chunk queued behind the first, so its request does not wait for the host
// (admissions, the other lane) between chunks; the small lane holds one,
// so that its slots can change at every chunk boundary.
struct LaneState {
    Chunk q[kDepth];
    int head = 0, n = 0;
    double step_ms = 0.0;         // recent wall time of one step (small lane)
    Chunk &oldest() { return q[head]; }
    int free_buf() const { return (head + n) % kDepth; }
};

static int run(dfpr_server *srv, dfpr_server_stats *st)
{
    std::vector<Slot> slots(srv->max_slots);
    std::vector<int> slot_lane(srv->max_slots, -1);
    std::vector<int64_t> order(srv->reqs.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = (int64_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return srv->reqs[a].arrival_ms < srv->reqs[b].arrival_ms;
    });
    // work already queued on a graph's own stream comes first; each graph
    // runs on its lane's stream while the server runs and gets its own
    // stream back at the end
    std::vector<hipStream_t> saved(srv->graphs.size());
    for (size_t i = 0; i < srv->graphs.size(); i++) {
        GraphEntry &ge = srv->graphs[i];
        if (hipStreamSynchronize(ge.g->stream) != hipSuccess)
            return set_error(DFPR_E_DEVICE, "stream synchronisation failed");
        saved[i] = ge.g->stream;
        ge.g->stream = srv->stream[ge.lane];
        ge.busy = 0;
    }
    int64_t pending = 0;          // requests of earlier runs keep their results
    for (const Request &q : srv->reqs) pending += q.state == 0;
    int64_t in_flight = 0, peak = srv->resident;
    size_t next = 0;              // first request of `order` not yet admitted
    int64_t done = 0, failed = 0;
    int32_t steps = 0, max_active = 0;
    uint32_t epochs = 0;
    LaneState lanes[kLanes];
    const Clock::time_point t0 = Clock::now();
    double last_done = 0.0;
    int rc = DFPR_OK;
    auto active_in = [&](int lane) {
        int k = 0;
        for (int i = 0; i < srv->max_slots; i++) k += slots[i].req >= 0 && slot_lane[i] == lane;
        return k;
    };
    auto launch = [&](int lane, std::vector<Slot *> &cs, int K) -> int {
        LaneState &L = lanes[lane];
        const int buf = L.free_buf();
        // small steps leave most of the GPU to a large request
        const uint32_t cap = lane == 1 && active_in(0) > 0 ? kSmallLaneBlocks : 0u;
        const int lrc = launch_chunk(srv, lane, buf, cs, K, cap);
        if (lrc) return lrc;
        Chunk &c = L.q[buf];
        c.cs = cs;
        c.epoch.clear();
        for (Slot *sl : cs) c.epoch.push_back(sl->epoch);
        c.K = K;
        c.buf = buf;
        c.t = Clock::now();
        L.n++;
        steps += K;
        return DFPR_OK;
    };
    while (done + failed < pending) {
        // 1. chunks for the lanes with admitted requests
        int active = 0;
        for (const Slot &s : slots) active += s.req >= 0;
        max_active = std::max(max_active, (int32_t)active);
        while (next < order.size() && srv->reqs[order[next]].state != 0) next++;
        const bool waiting = next < order.size() && active < srv->max_slots;
        for (int lane = 0; lane < kLanes; lane++) {
            LaneState &L = lanes[lane];
            std::vector<Slot *> cs;
            for (int i = 0; i < srv->max_slots; i++)
                if (slots[i].req >= 0 && slot_lane[i] == lane) cs.push_back(&slots[i]);
            if (cs.empty()) continue;
            if (L.n == 0) {
                int K = kMaxChunk;
                for (Slot *s : cs) K = std::min(K, s->pred);
                // requests join the small lane at chunk boundaries: keep its
                // chunks short while a slot is free and requests are still to come
                if (lane == 1 && waiting && L.step_ms > 0.0)
                    K = std::min(K, std::max(1, (int)(kChunkMsWhileWaiting / L.step_ms)));
                rc = launch(lane, cs, std::max(K, 1));
                if (rc) goto out;
            }
            if (lane == 0 && L.n == 1) {
                // the iterations predicted beyond those queued, and at least
                // two more, so that the device has work while the host looks
                Slot *s = cs[0];
                const int K = std::min(kMaxChunk, std::max(2, s->pred - (s->itq - s->it)));
                rc = launch(lane, cs, K);
                if (rc) goto out;
            }
        }
        // 2. admission in arrival order, overlapping the chunks; a request
        // whose graph is busy, or whose lane is full, waits without blocking
        // later ones; the budget is first come, first served
        {
            int admitted = 0;
            double now = ms_since(t0);
            auto view = [&](int64_t r) {
                const Request &q = srv->reqs[r];
                return PendingView{q.arrival_ms, q.state, q.gid, q.charge};
            };
            auto blocked = [&](int32_t gid) {
                const GraphEntry &ge = srv->graphs[gid];
                return ge.busy != 0 || (ge.lane == 0 && active_in(0) > 0);
            };
            for (size_t from = next;;) {
                auto free_slot = std::find_if(slots.begin(), slots.end(),
                                              [](const Slot &s) { return s.req < 0; });
                const int64_t pos = next_admission(order, from, now, free_slot != slots.end(), view,
                                                   blocked, srv->resident + in_flight, srv->budget);
                if (pos < 0) break;
                from = (size_t)pos + 1;
                Request &q = srv->reqs[order[(size_t)pos]];
                srv->graphs[q.gid].busy = 1;
                in_flight += q.charge;
                peak = std::max(peak, srv->resident + in_flight);
                const size_t si = (size_t)(free_slot - slots.begin());
                slot_lane[si] = srv->graphs[q.gid].lane;
                const int arc = admit(srv, order[(size_t)pos], *free_slot, now);
                if (arc) {
                    // a rejected batch leaves its graph unchanged
                    q.state = 2;
                    q.res.status = arc;
                    q.res.done_ms = ms_since(t0);
                    free_slot->req = -1;
                    srv->graphs[q.gid].busy = 0;
                    in_flight -= q.charge;
                    failed++;
                    if (arc != DFPR_E_RANGE) {
                        rc = arc;
                        goto out;
                    }
                } else {
                    free_slot->epoch = ++epochs;
                    admitted++;
                }
                now = ms_since(t0);
            }
            // a new request may start a chunk on an idle lane at once
            if (admitted) {
                bool idle = false;
                for (int lane = 0; lane < kLanes; lane++)
                    idle |= lanes[lane].n == 0 && active_in(lane) > 0;
                if (idle) continue;
            }
        }
        bool any_busy = false;
        for (const LaneState &L : lanes) any_busy |= L.n > 0;
        if (!any_busy) {
            while (next < order.size() && srv->reqs[order[next]].state != 0) next++;
            if (next < order.size()) {
                const double wait = srv->reqs[order[next]].arrival_ms - ms_since(t0);
                if (wait > 0.05)
                    std::this_thread::sleep_for(std::chrono::duration<double, std::milli>(
                        std::min(wait, 1.0)));
            }
            continue;
        }
        // 3. the results of the first lane to finish its oldest chunk; while
        // the lanes run, look for arrivals that could take a free slot
        int lane = -1;
        while (lane < 0) {
            for (int l = 0; l < kLanes && lane < 0; l++) {
                if (lanes[l].n == 0) continue;
                const hipError_t e = hipEventQuery(srv->done[l][lanes[l].oldest().buf]);
                if (e == hipSuccess) lane = l;
                else if (e != hipErrorNotReady) {
                    rc = set_error(DFPR_E_DEVICE, "stream synchronisation failed");
                    goto out;
                }
            }
            if (lane >= 0) break;
            while (next < order.size() && srv->reqs[order[next]].state != 0) next++;
            int act = 0;
            for (const Slot &s : slots) act += s.req >= 0;
            if (next < order.size() && act < srv->max_slots &&
                srv->reqs[order[next]].arrival_ms <= ms_since(t0)) {
                // an arrival could start now: admit it before waiting more
                // (its lane may be idle)
                break;
            }
            std::this_thread::yield();
        }
        if (lane < 0) continue;
        {
            LaneState &L = lanes[lane];
            Chunk ch = L.oldest();
            L.head = (L.head + 1) % kDepth;
            L.n--;
            if (lane == 1) {
                const double chunk_ms =
                    std::chrono::duration<double, std::milli>(Clock::now() - ch.t).count();
                const double per = chunk_ms / ch.K;
                L.step_ms = L.step_ms > 0.0 ? 0.5 * L.step_ms + 0.5 * per : per;
            }
            const Ctl *pin = srv->ctl_pin[lane][ch.buf];
            std::vector<Slot *> fin;
            std::vector<Ctl> fin_ctl;
            for (size_t i = 0; i < ch.cs.size(); i++) {
                Slot &s = *ch.cs[i];
                // a slot retired or moved to its next phase by an earlier
                // chunk only ran steps that returned at once here
                if (s.req < 0 || s.epoch != ch.epoch[i]) continue;
                Request &q = srv->reqs[s.req];
                GraphEntry &ge = srv->graphs[q.gid];
                dfpr_graph *g = ge.g;
                const Ctl c = pin[i];
                *g->ctl_host = c;
                s.it = c.iterations;
                const int res = s.base ^ ((c.iterations - s.it0) & 1);
                if (c.err) {
                    q.res.status = DFPR_E_RANGE;
                    fin.push_back(&s);
                    continue;
                }
                if (s.phase32 && (c.phase_end || c.done)) {
                    rc = df_phase_end(g, res, c.done != 0);
                    if (rc) goto out;
                    if (!c.done) {
                        s.phase32 = 0;
                        s.it0 = c.iterations;
                        s.itq = c.iterations;
                        s.epoch = ++epochs;
                        s.base = res;
                        s.prev_dr = -1.0;
                        s.pred = 2;
                        q.res.refine_sweeps = -c.iterations;   // completed at retirement
                        continue;
                    }
                }
                if (c.done) {
                    rc = df_finish(g, s.sbase, res, c.iterations);
                    if (rc) goto out;
                    fin.push_back(&s);
                    continue;
                }
                predict(s, c, ge.p.tol);
            }
            if (!fin.empty()) {
                // the lane's later chunk, if any, only has steps of finished
                // slots that return at once (the large lane holds one slot),
                // so waiting for the stream is short
                CtlGather cg{};
                cg.n = (int32_t)fin.size();
                for (size_t i = 0; i < fin.size(); i++)
                    cg.src[i] = srv->graphs[srv->reqs[fin[i]->req].gid].g->ctl;
                cg.dst = srv->ctl_dev[lane][ch.buf];
                k_gather_ctl<<<1, kBlock, 0, srv->stream[lane]>>>(cg);
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(srv->ctl_pin[lane][ch.buf], srv->ctl_dev[lane][ch.buf],
                                   fin.size() * sizeof(Ctl), hipMemcpyDeviceToHost,
                                   srv->stream[lane]) != hipSuccess ||
                    hipStreamSynchronize(srv->stream[lane]) != hipSuccess) {
                    rc = set_error(DFPR_E_DEVICE, "finishing failed on the device");
                    goto out;
                }
                const double t = ms_since(t0);
                for (size_t i = 0; i < fin.size(); i++) {
                    Slot &s = *fin[i];
                    Request &q = srv->reqs[s.req];
                    GraphEntry &ge = srv->graphs[q.gid];
                    const Ctl &c = srv->ctl_pin[lane][ch.buf][i];
                    *ge.g->ctl_host = c;
                    q.state = 2;
                    q.res.done_ms = t;
                    if (q.res.status == DFPR_OK) {
                        q.res.iterations = c.iterations;
                        q.res.converged = c.converged;
                        q.res.final_linf = c.final_linf;
                        q.res.edges_processed = (int64_t)c.edges;
                        q.res.affected = (int64_t)c.affected;
                        q.res.refine_sweeps =
                            q.res.refine_sweeps < 0 ? c.iterations + q.res.refine_sweeps : 0;
                        done++;
                    } else {
                        failed++;
                    }
                    last_done = t;
                    ge.busy = 0;
                    in_flight -= q.charge;
                    s = Slot();
                }
            }
        }
    }
out:
    if (rc) {
        for (int l = 0; l < kLanes; l++) (void)hipStreamSynchronize(srv->stream[l]);
        (void)hipStreamSynchronize(srv->astream);
        // requests in flight end with the run's error; later runs do not
        // take them up again
        for (Slot &s : slots) {
            if (s.req < 0) continue;
            Request &q = srv->reqs[s.req];
            q.state = 2;
            q.res.status = rc;
            q.res.done_ms = ms_since(t0);
            srv->graphs[q.gid].busy = 0;
            s = Slot();
        }
    }
    for (size_t i = 0; i < srv->graphs.size(); i++) srv->graphs[i].g->stream = saved[i];
    if (rc) return rc;
    if (st) {
        std::vector<double> lat, queue;
        for (const Request &q : srv->reqs) {
            if (q.res.status != DFPR_OK || q.state != 2) continue;
            lat.push_back(q.res.done_ms - q.res.arrival_ms);
            queue.push_back(q.res.admit_ms - q.res.arrival_ms);
        }
        double sum = 0.0;
        for (double x : lat) sum += x;
        st->requests = (int64_t)srv->reqs.size();
        st->completed = done;
        st->failed = failed;
        st->wall_ms = last_done;
        st->updates_per_s = last_done > 0 ? done / (last_done / 1e3) : 0.0;
        st->latency_p50_ms = pct(lat, 50);
        st->latency_p99_ms = pct(lat, 99);
        st->latency_mean_ms = lat.empty() ? 0.0 : sum / lat.size();
        st->queue_p50_ms = pct(queue, 50);
        st->queue_p99_ms = pct(queue, 99);
        st->max_active = max_active;
        st->steps = steps;
        st->peak_bytes = peak;
    }
    return DFPR_OK;
}

}  // namespace dfpr

extern "C" {

int dfpr_server_create(int32_t max_slots, int64_t hbm_budget_bytes, dfpr_server **out)
{
    if (!out) return set_error(DFPR_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > kMaxSlots || hbm_budget_bytes <= 0)
        return set_error(DFPR_E_ARG, "need 1 <= max_slots <= 8 and a positive budget");
    dfpr_server *s = new dfpr_server();
    s->max_slots = max_slots;
    s->budget = hbm_budget_bytes;
    hipError_t e = hipStreamCreateWithFlags(&s->astream, hipStreamNonBlocking);
    for (int l = 0; l < kLanes; l++) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream[l], hipStreamNonBlocking);
        for (int b = 0; b < kDepth; b++) {
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&s->done[l][b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipMalloc(&s->ctl_dev[l][b], kMaxSlots * sizeof(Ctl));
            if (e == hipSuccess) e = hipHostMalloc(&s->ctl_pin[l][b], kMaxSlots * sizeof(Ctl));
        }
    }
    if (e != hipSuccess) {
        dfpr_server_free(s);
        return hip_fail(e, "server set-up");
    }
    *out = s;
    return DFPR_OK;
}

void dfpr_server_free(dfpr_server *s)
{
    if (!s) return;
    for (hipStream_t st : {s->stream[0], s->stream[1], s->astream})
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    for (int l = 0; l < kLanes; l++)
        for (int b = 0; b < kDepth; b++) {
            if (s->done[l][b]) (void)hipEventDestroy(s->done[l][b]);
            (void)hipFree(s->ctl_dev[l][b]);
            (void)hipHostFree(s->ctl_pin[l][b]);
        }
    delete s;
}

int dfpr_server_set_large_edges(dfpr_server *s, int64_t large_edges)
{
    if (!s || large_edges < 1) return set_error(DFPR_E_ARG, "need a server and large_edges >= 1");
    s->large_edges = large_edges;
    for (GraphEntry &ge : s->graphs) ge.lane = ge.g->m >= large_edges ? 0 : 1;
    return DFPR_OK;
}

int dfpr_server_add_graph(dfpr_server *s, dfpr_graph *g, const dfpr_params *p, int32_t *graph_id)
{
    if (!s || !g) return set_error(DFPR_E_ARG, "NULL argument");
    GraphEntry ge;
    int rc = check_params(p, ge.p);
    if (rc) return rc;
    for (const GraphEntry &x : s->graphs)
        if (x.g == g) return set_error(DFPR_E_ARG, "graph already added");
    ge.g = g;
    ge.bytes = graph_bytes(g);
    ge.lane = g->m >= s->large_edges ? 0 : 1;
    if (s->resident + ge.bytes > s->budget)
        return set_error(DFPR_E_NOMEM, "resident graphs exceed the HBM budget");
    DFPR_HIP(hipStreamSynchronize(g->stream));
    s->resident += ge.bytes;
    s->graphs.push_back(ge);
    if (graph_id) *graph_id = (int32_t)s->graphs.size() - 1;
    return DFPR_OK;
}

int dfpr_server_submit(dfpr_server *s, int32_t graph_id, double arrival_ms, int64_t n_del,
                       const int32_t *del_src, const int32_t *del_dst, int64_t n_ins,
                       const int32_t *ins_src, const int32_t *ins_dst, int64_t *request_id)
{
    if (!s || graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
        return set_error(DFPR_E_ARG, "unknown graph");
    if (n_del < 0 || n_ins < 0 || (n_del && (!del_src || !del_dst)) ||
        (n_ins && (!ins_src || !ins_dst)) || !(arrival_ms >= 0.0))
        return set_error(DFPR_E_ARG, "bad request");
    Request q;
    q.gid = graph_id;
    q.arrival_ms = arrival_ms;
    q.ds.assign(del_src, del_src + n_del);
    q.dd.assign(del_dst, del_dst + n_del);
    q.is.assign(ins_src, ins_src + n_ins);
    q.id.assign(ins_dst, ins_dst + n_ins);
    q.charge = kRequestBytesPerEntry * (n_del + n_ins);
    if (s->resident + q.charge > s->budget)
        return set_error(DFPR_E_NOMEM, "request can never fit the HBM budget");
    q.res.graph_id = graph_id;
    q.res.arrival_ms = arrival_ms;
    s->reqs.push_back(std::move(q));
    if (request_id) *request_id = (int64_t)s->reqs.size() - 1;
    return DFPR_OK;
}

int dfpr_server_run(dfpr_server *s, dfpr_server_stats *st)
{
    if (!s) return set_error(DFPR_E_ARG, "server is NULL");
    for (GraphEntry &ge : s->graphs)
        if (__atomic_exchange_n(&ge.g->busy, 1, __ATOMIC_ACQ_REL)) {
            for (GraphEntry &x : s->graphs) {
                if (&x == &ge) break;
                __atomic_store_n(&x.g->busy, 0, __ATOMIC_RELEASE);
            }
            return set_error(DFPR_E_BUSY, "a graph is in use");
        }
    const int rc = run(s, st);
    for (GraphEntry &ge : s->graphs) __atomic_store_n(&ge.g->busy, 0, __ATOMIC_RELEASE);
    return rc;
}

int dfpr_server_result(const dfpr_server *s, int64_t request_id, dfpr_request_result *out)
{
    if (!s || !out || request_id < 0 || request_id >= (int64_t)s->reqs.size())
        return set_error(DFPR_E_ARG, "unknown request");
    *out = s->reqs[request_id].res;
    return DFPR_OK;
}

}  // extern "C"
