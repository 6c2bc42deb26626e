// Admission rule of the serving loop (serve.hip), host code only, so that
// it can be tested without a device.  A request may start when it has
// arrived, a slot is free, no other update of its graph is in flight (one
// writer per graph, Section 3.2) and the HBM budget has room for its
// charge.  Requests are considered in arrival order; the budget is first
// come, first served (a request that does not fit stops the scan, so later
// small requests cannot starve it), while a request whose graph is busy
// is passed over without blocking requests for other graphs.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace dfpr {

struct PendingView {
    double arrival_ms;   // arrival time, relative to the start of the run
    int state;           // 0 waiting, 1 running, 2 done
    int32_t gid;         // graph the request updates
    int64_t charge;      // bytes it holds while in flight
};

// Position in `order` (scanned from `from`) of the next request to admit
// at time `now`, or -1.  `view(r)` describes request r; `graph_busy(g)`
// tells whether graph g has an update in flight; `used` is the budget
// already taken (resident graphs and requests in flight).
template <class View, class Busy>
int64_t next_admission(const std::vector<int64_t> &order, size_t from, double now,
                       bool slot_free, const View &view, const Busy &graph_busy, int64_t used,
                       int64_t budget)
{
    if (!slot_free) return -1;
    for (size_t k = from; k < order.size(); k++) {
        const PendingView q = view(order[k]);
        if (q.state != 0) continue;
        if (q.arrival_ms > now) return -1;
        if (graph_busy(q.gid)) continue;
        if (used + q.charge > budget) return -1;
        return (int64_t)k;
    }
    return -1;
}

}  // namespace dfpr
