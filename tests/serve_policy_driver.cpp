// Drives the serving loop's admission rule (serve_policy.h) with a fake
// clock and a mock budget, no device: arrival order, requests that have not
// arrived, one writer per graph, first-come budget, no free slot, and a
// full run of a queue through a fixed number of slots.  Built and run by
// test_serve_policy.py; prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <vector>

#include "serve_policy.h"

using dfpr::PendingView;
using dfpr::next_admission;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                         \
        }                                                                     \
    } while (0)

struct World {
    std::vector<PendingView> reqs;
    std::vector<int64_t> order;      // by arrival (stable)
    std::vector<char> busy;          // per graph
    int64_t next(size_t from, double now, bool slot, int64_t used, int64_t budget) const
    {
        auto view = [&](int64_t r) { return reqs[r]; };
        auto gb = [&](int32_t g) { return busy[g] != 0; };
        return next_admission(order, from, now, slot, view, gb, used, budget);
    }
};

int main()
{
    World w;
    // request: arrival, state, graph, charge
    w.reqs = {{0.0, 0, 0, 10}, {1.0, 0, 0, 10}, {1.0, 0, 1, 50}, {2.0, 0, 2, 10}, {5.0, 0, 1, 10}};
    w.order = {0, 1, 2, 3, 4};
    w.busy = {0, 0, 0};

    // arrival order; nothing that has not arrived
    CHECK(w.next(0, 0.0, true, 0, 1000) == 0);
    CHECK(w.next(1, 0.5, true, 0, 1000) == -1);
    // no free slot: nothing
    CHECK(w.next(0, 10.0, false, 0, 1000) == -1);
    // one writer: request 1 waits for graph 0, request 2 (graph 1) goes first
    w.busy[0] = 1;
    CHECK(w.next(1, 1.0, true, 0, 1000) == 2);
    // the budget is first come, first served: request 2 (50 bytes) does
    // not fit, so request 3 behind it is not admitted either
    CHECK(w.next(1, 2.0, true, 960, 1000) == -1);
    CHECK(w.next(1, 2.0, true, 950, 1000) == 2);
    // requests already running or done are skipped
    w.reqs[2].state = 1;
    CHECK(w.next(1, 2.0, true, 0, 1000) == 3);
    w.busy[0] = 0;
    CHECK(w.next(1, 2.0, true, 0, 1000) == 1);

    // a full run: two slots, a fake clock in 1 ms steps, each admitted
    // request finishing 3 ms later; every request completes, at most two
    // run at once, never two of one graph, none before its arrival, and
    // the budget is never exceeded
    World r;
    const int N = 40;
    for (int i = 0; i < N; i++)
        r.reqs.push_back({0.5 * i, 0, (int32_t)(i % 3), (int64_t)(10 + 7 * (i % 5))});
    for (int i = 0; i < N; i++) r.order.push_back(i);
    r.busy.assign(3, 0);
    const int64_t budget = 100;
    std::vector<double> end(N, -1.0), start(N, -1.0);
    int running = 0, done = 0;
    int64_t used = 0;
    for (int t = 0; t < 1000 && done < N; t++) {
        const double now = t;
        for (int i = 0; i < N; i++)
            if (r.reqs[i].state == 1 && end[i] <= now) {
                r.reqs[i].state = 2;
                r.busy[r.reqs[i].gid] = 0;
                used -= r.reqs[i].charge;
                running--;
                done++;
            }
        for (size_t from = 0;;) {
            const int64_t pos = r.next(from, now, running < 2, used, budget);
            if (pos < 0) break;
            const int64_t q = r.order[(size_t)pos];
            CHECK(r.reqs[q].arrival_ms <= now && !r.busy[r.reqs[q].gid]);
            r.reqs[q].state = 1;
            r.busy[r.reqs[q].gid] = 1;
            used += r.reqs[q].charge;
            CHECK(used <= budget);
            running++;
            CHECK(running <= 2);
            start[q] = now;
            end[q] = now + 3.0;
            from = (size_t)pos + 1;
        }
    }
    CHECK(done == N);
    // one graph's requests start in arrival order
    for (int i = 0; i < N; i++)
        for (int j = i + 1; j < N; j++)
            if (r.reqs[i].gid == r.reqs[j].gid) CHECK(start[i] <= start[j]);
    std::printf("ok\n");
    return 0;
}
