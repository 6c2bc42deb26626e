// Serving form: continuous batching of Dynamic Frontier updates over many
// resident graphs.
//
// Graphs stay resident on the device with their ranks.  Update requests
// (graph, batch, arrival time) wait in arrival order and are admitted into
// one of a few slots when (a) a slot is free, (b) their graph has no update
// in flight (one writer per graph, Section 3.2) and (c) the HBM budget
// covers the resident graphs plus the scratch of every admitted request.
// Admission applies the batch to the graph and runs the initial marking.
// Every step then runs one iteration of every admitted request in one
// coalesced launch: the workgroups are split among the slots in proportion
// to the work each can use, so small and large graphs share the device.
// After each step a request whose iteration loop ended is retired and its
// slot is free for the next arrival, so requests join and leave at
// iteration boundaries rather than waiting for a whole batch to finish.
//
// Each slot runs exactly the per-row code of the single-graph engine
// (iter.h) with the same class of every row, so a request's result does not
// depend on what else is in flight.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "common.h"
#include "iter.h"

namespace dfpr {

constexpr int kMaxSlots = 8;
constexpr int64_t kRequestBytesPerEntry = 96;   // device scratch per batch entry

struct MultiArgs {
    int32_t nslots;
    uint32_t grid;            // workgroups shared by the slots
    uint32_t *active_out;     // per slot: workgroups that wrote partials
    IterArgs s[kMaxSlots];
};
static_assert(sizeof(MultiArgs) <= 4096, "kernel arguments must fit in 4 KiB");

// Split m.grid workgroups among the slots in proportion to the workgroups
// each can use; a slot whose loop has ended gets none.  Every workgroup
// computes the same split.
template <bool F32>
__device__ inline void split_grid(const MultiArgs &m, Plan &tmp, uint32_t *start,
                                  uint32_t *alloc, uint32_t *active)
{
    uint32_t demand[kMaxSlots];
    uint64_t total = 0;
    for (int s = 0; s < m.nslots; s++) {
        const IterArgs &a = m.s[s];
        const Ctl *c = a.ctl;
        demand[s] = 0;
        if (c->done || (F32 && c->phase_end)) continue;
        make_plan(a, c, !c->dense, a.it & 1, tmp);
        demand[s] = active_blocks(tmp, m.grid);
        total += demand[s];
    }
    uint32_t at = 0;
    for (int s = 0; s < m.nslots; s++) {
        uint32_t g = demand[s];
        if (g && total > m.grid) g = max(1u, (uint32_t)((uint64_t)demand[s] * m.grid / total));
        start[s] = at;
        alloc[s] = g;
        active[s] = 0;
        if (g) {
            const IterArgs &a = m.s[s];
            make_plan(a, a.ctl, !a.ctl->dense, a.it & 1, tmp);
            active[s] = active_blocks(tmp, g);
        }
        at += g;
    }
    start[m.nslots] = at;
}

template <bool F32>
__global__ __launch_bounds__(kBlock) void k_iter_multi(MultiArgs m)
{
    __shared__ IterShared sh;
    __shared__ uint32_t s_start[kMaxSlots + 1], s_alloc[kMaxSlots], s_active[kMaxSlots];
    if (threadIdx.x == 0) {
        split_grid<F32>(m, sh.plan, s_start, s_alloc, s_active);
        if (blockIdx.x == 0)
            for (int s = 0; s < m.nslots; s++) m.active_out[s] = s_active[s];
    }
    __syncthreads();
    int slot = -1;
    for (int s = 0; s < m.nslots; s++)
        if (blockIdx.x >= s_start[s] && blockIdx.x < s_start[s + 1]) slot = s;
    if (slot < 0) return;
    iter_body<true, F32>(m.s[slot], blockIdx.x - s_start[slot], s_alloc[slot], sh);
}

// One workgroup per slot.
template <bool F32>
__global__ __launch_bounds__(kBlock) void k_final_multi(MultiArgs m)
{
    __shared__ IterShared sh;
    const int s = blockIdx.x;
    if (s >= m.nslots || m.active_out[s] == 0) return;
    final_body(m.s[s], m.active_out[s], true, F32, sh);
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
    int it = 0;               // next iteration
};

struct GraphEntry {
    dfpr_graph *g = nullptr;
    dfpr_params p{};
    int64_t bytes = 0;
    int busy = 0;
};

// Device bytes a graph holds (CSRs, rank and contribution buffers, marks,
// class lists and schedule).
static int64_t graph_bytes(const dfpr_graph *g)
{
    const int64_t n = g->n;
    int64_t b = 0;
    for (int o = 0; o < 2; o++) b += (int64_t)g->csr[o].slots * 4 + 3 * n * 4;
    b += 4 * n * 8 + 2 * n * 4 + 2 * n * 4 + (int64_t)kBins * n * 4 + n * 4;
    return b;
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
    int64_t budget = 0;
    int64_t resident = 0;
    std::vector<dfpr::GraphEntry> graphs;
    std::vector<dfpr::Request> reqs;
    hipStream_t stream = nullptr;
    uint32_t *active_dev = nullptr;   // 2 x kMaxSlots
    int grid = 1024;
};

using namespace dfpr;

namespace dfpr {

static double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Admit request r into slot sl: apply the batch, then begin the update.
static int admit(dfpr_server *srv, int64_t r, Slot &sl, double now_ms)
{
    Request &q = srv->reqs[r];
    GraphEntry &ge = srv->graphs[q.gid];
    dfpr_graph *g = ge.g;
    q.state = 1;
    q.res.admit_ms = now_ms;
    int64_t applied[2] = {0, 0};
    const int64_t nd = (int64_t)q.ds.size(), ni = (int64_t)q.is.size();
    int rc = apply_batch_impl(g, nd, q.ds.data(), q.dd.data(), ni, q.is.data(), q.id.data(), 0,
                              applied);
    if (rc) return rc;
    q.res.applied[0] = applied[0];
    q.res.applied[1] = applied[1];
    const int32_t *bds, *bdd, *bis, *bid;
    rc = stage_batch(g, nd, q.ds.data(), q.dd.data(), ni, q.is.data(), q.id.data(), &bds, &bdd,
                     &bis, &bid);
    if (rc) return rc;
    uint32_t sbase = 0;
    rc = df_begin(g, ge.p, nd, bds, bdd, ni, bis, bid, nullptr, 0, &sbase);
    if (rc) return rc;
    sl.req = r;
    sl.sbase = sbase;
    sl.phase32 = ge.p.precision == DFPR_FP32_KAHAN ? 1 : 0;
    sl.it0 = 0;
    sl.base = g->cur;
    sl.it = 0;
    return DFPR_OK;
}

// One coalesced iteration of every slot in the given phase.
static int launch_group(dfpr_server *srv, std::vector<Slot> &slots, bool f32)
{
    MultiArgs m{};
    m.grid = (uint32_t)srv->grid;
    m.active_out = srv->active_dev + (f32 ? kMaxSlots : 0);
    for (Slot &sl : slots) {
        if (sl.req < 0 || (sl.phase32 != 0) != f32) continue;
        const Request &q = srv->reqs[sl.req];
        GraphEntry &ge = srv->graphs[q.gid];
        dfpr_graph *g = ge.g;
        IterArgs a = iter_args(g, ge.p, sl.sbase);
        const int src = sl.base ^ ((sl.it - sl.it0) & 1);
        a.Rc = g->R[src];
        a.Cc = g->C[src];
        a.Rn = g->R[src ^ 1];
        a.Cn = g->C[src ^ 1];
        a.C32c = g->C32[src];
        a.C32n = g->C32[src ^ 1];
        a.it = sl.it;
        m.s[m.nslots++] = a;
    }
    if (!m.nslots) return DFPR_OK;
    if (f32) {
        k_iter_multi<true><<<m.grid + kMaxSlots, kBlock, 0, srv->stream>>>(m);
        k_final_multi<true><<<m.nslots, kBlock, 0, srv->stream>>>(m);
    } else {
        k_iter_multi<false><<<m.grid + kMaxSlots, kBlock, 0, srv->stream>>>(m);
        k_final_multi<false><<<m.nslots, kBlock, 0, srv->stream>>>(m);
    }
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
}

static int run(dfpr_server *srv, dfpr_server_stats *st)
{
    std::vector<Slot> slots(srv->max_slots);
    std::vector<int64_t> order(srv->reqs.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = (int64_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return srv->reqs[a].arrival_ms < srv->reqs[b].arrival_ms;
    });
    // work already queued on a graph's own stream comes first; the server
    // stream carries every graph while it runs and the graphs get their
    // streams back at the end
    std::vector<hipStream_t> saved(srv->graphs.size());
    for (size_t i = 0; i < srv->graphs.size(); i++) {
        GraphEntry &ge = srv->graphs[i];
        if (hipStreamSynchronize(ge.g->stream) != hipSuccess)
            return set_error(DFPR_E_DEVICE, "stream synchronisation failed");
        saved[i] = ge.g->stream;
        ge.g->stream = srv->stream;
        ge.busy = 0;
    }
    int64_t pending = 0;          // requests of earlier runs keep their results
    for (const Request &q : srv->reqs) pending += q.state == 0;
    int64_t in_flight = 0, peak = srv->resident;
    size_t next = 0;              // first request of `order` not yet admitted
    int64_t done = 0, failed = 0;
    int32_t steps = 0, max_active = 0;
    const Clock::time_point t0 = Clock::now();
    double last_done = 0.0;
    int rc = DFPR_OK;
    while (done + failed < pending) {
        // admission in arrival order; a request whose graph is busy waits
        // without blocking later ones; the budget is first come, first served
        double now = ms_since(t0);
        for (size_t k = next; k < order.size(); k++) {
            Request &q = srv->reqs[order[k]];
            if (q.state != 0) continue;
            if (q.arrival_ms > now) break;
            auto free_slot = std::find_if(slots.begin(), slots.end(),
                                          [](const Slot &s) { return s.req < 0; });
            if (free_slot == slots.end()) break;
            if (srv->graphs[q.gid].busy) continue;
            if (srv->resident + in_flight + q.charge > srv->budget) break;
            srv->graphs[q.gid].busy = 1;
            in_flight += q.charge;
            peak = std::max(peak, srv->resident + in_flight);
            int arc = admit(srv, order[k], *free_slot, now);
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
            }
            now = ms_since(t0);
        }
        while (next < order.size() && srv->reqs[order[next]].state != 0) next++;
        int active = 0;
        for (const Slot &s : slots) active += s.req >= 0;
        if (!active) {
            if (next < order.size()) {
                const double wait = srv->reqs[order[next]].arrival_ms - ms_since(t0);
                if (wait > 0.05)
                    std::this_thread::sleep_for(std::chrono::duration<double, std::milli>(
                        std::min(wait, 1.0)));
            }
            continue;
        }
        max_active = std::max(max_active, active);
        // one iteration of every admitted request
        rc = launch_group(srv, slots, false);
        if (!rc) rc = launch_group(srv, slots, true);
        if (rc) goto out;
        steps++;
        for (const Slot &s : slots) {
            if (s.req < 0) continue;
            dfpr_graph *g = srv->graphs[srv->reqs[s.req].gid].g;
            if (hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                               srv->stream) != hipSuccess) {
                rc = set_error(DFPR_E_DEVICE, "control block copy failed");
                goto out;
            }
        }
        if (hipStreamSynchronize(srv->stream) != hipSuccess) {
            rc = set_error(DFPR_E_DEVICE, "stream synchronisation failed");
            goto out;
        }
        bool finishing = false;
        for (Slot &s : slots) {
            if (s.req < 0) continue;
            Request &q = srv->reqs[s.req];
            GraphEntry &ge = srv->graphs[q.gid];
            dfpr_graph *g = ge.g;
            const Ctl c = *g->ctl_host;
            s.it = c.iterations;
            const int res = s.base ^ ((c.iterations - s.it0) & 1);
            if (c.err) {
                q.res.status = DFPR_E_RANGE;
                q.state = 3;       // retire without results
                finishing = true;
                continue;
            }
            if (s.phase32 && (c.phase_end || c.done)) {
                rc = df_phase_end(g, res, c.done != 0);
                if (rc) goto out;
                if (!c.done) {
                    s.phase32 = 0;
                    s.it0 = c.iterations;
                    s.base = res;
                    q.res.refine_sweeps = -c.iterations;   // completed at retirement
                    continue;
                }
            }
            if (c.done) {
                rc = df_finish(g, s.sbase, res, c.iterations);
                if (rc) goto out;
                if (hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                                   srv->stream) != hipSuccess) {
                    rc = set_error(DFPR_E_DEVICE, "control block copy failed");
                    goto out;
                }
                q.state = 3;
                finishing = true;
            }
        }
        if (finishing) {
            if (hipStreamSynchronize(srv->stream) != hipSuccess) {
                rc = set_error(DFPR_E_DEVICE, "stream synchronisation failed");
                goto out;
            }
            const double t = ms_since(t0);
            for (Slot &s : slots) {
                if (s.req < 0 || srv->reqs[s.req].state != 3) continue;
                Request &q = srv->reqs[s.req];
                GraphEntry &ge = srv->graphs[q.gid];
                const Ctl &c = *ge.g->ctl_host;
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
                s.req = -1;
            }
        }
    }
out:
    if (rc) (void)hipStreamSynchronize(srv->stream);
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
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&s->active_dev, 2 * kMaxSlots * sizeof(uint32_t));
    if (e != hipSuccess) {
        dfpr_server_free(s);
        return hip_fail(e, "server set-up");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) == hipSuccess && prop.multiProcessorCount > 0)
        s->grid = std::min(kMaxGrid - kMaxSlots, prop.multiProcessorCount * 8);
    *out = s;
    return DFPR_OK;
}

void dfpr_server_free(dfpr_server *s)
{
    if (!s) return;
    if (s->stream) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipStreamDestroy(s->stream);
    }
    (void)hipFree(s->active_dev);
    delete s;
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
