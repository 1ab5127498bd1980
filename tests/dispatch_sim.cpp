// Host-only driver of the served stream's dispatch policy (dispatch.h) for
// tests: a simulated clock and a fake executor in place of the device.  A
// launched batch keeps its lane busy for a + b * hits seconds.
//
// Scenario on stdin, one directive per line:
//   deadline D          seconds an event may wait while other lanes run
//   queue_limit Q       pending events before submit refuses
//   service A B         batch time = A + B * hits
//   lane G E H          a lane of grid G with E event slots and a pool of H hits
//   event T G N         an event of N hits for grid G arriving at time T (in order)
//   stop T              the server starts stopping at time T
// Log on stdout, one line per step:
//   launch T LANE GRID ID...   |  done T LANE  |  refuse T ID never_fits|queue_full
//   end T                      (everything finished)  |  stuck T
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "dispatch.h"

using hough::serve::Admit;
using hough::serve::LaneState;

struct Ev {
    int id;
    double t;
    int grid;
    int64_t hits;
};

int main() {
    double deadline = 0.002, svc_a = 0.0, svc_b = 0.0, stop_at = INFINITY;
    int64_t queue_limit = 4096;
    std::vector<LaneState> lanes;
    std::vector<Ev> arrivals;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string what;
        if (!(in >> what))
            continue;
        if (what == "deadline") {
            in >> deadline;
        } else if (what == "queue_limit") {
            in >> queue_limit;
        } else if (what == "service") {
            in >> svc_a >> svc_b;
        } else if (what == "lane") {
            LaneState l{};
            in >> l.grid >> l.max_events >> l.max_hits;
            l.busy = false;
            lanes.push_back(l);
        } else if (what == "event") {
            Ev e{};
            e.id = static_cast<int>(arrivals.size());
            in >> e.t >> e.grid >> e.hits;
            arrivals.push_back(e);
        } else if (what == "stop") {
            in >> stop_at;
        }
    }
    int n_grids = 0;
    for (const auto &l : lanes)
        n_grids = std::max(n_grids, l.grid + 1);
    std::vector<std::deque<Ev>> q(n_grids);
    std::vector<int64_t> pending_hits(n_grids, 0), qlen(n_grids, 0);
    std::vector<double> busy_until(lanes.size(), 0.0);
    std::vector<int64_t> pool(n_grids, 0);
    for (const auto &l : lanes)
        pool[l.grid] = l.max_hits;
    int64_t n_pending = 0;
    size_t next = 0;
    double now = 0.0, wake = -1.0;
    bool stop = false;
    for (int guard = 0; guard < 10000000; ++guard) {
        for (size_t k = 0; k < lanes.size(); ++k)
            if (lanes[k].busy && busy_until[k] <= now) {
                lanes[k].busy = false;
                std::printf("done %.9f %zu\n", now, k);
            }
        while (next < arrivals.size() && arrivals[next].t <= now) {
            const Ev &e = arrivals[next++];
            const bool known = e.grid >= 0 && e.grid < n_grids;
            const Admit a = known ? hough::serve::admit(e.hits, pool[e.grid], false, n_pending, queue_limit)
                                  : Admit::never_fits;
            if (a == Admit::ok) {
                q[e.grid].push_back(e);
                pending_hits[e.grid] += e.hits;
                ++n_pending;
            } else {
                std::printf("refuse %.9f %d %s\n", now, e.id, a == Admit::never_fits ? "never_fits" : "queue_full");
            }
        }
        if (now >= stop_at)
            stop = true;
        while (true) {
            for (int g = 0; g < n_grids; ++g)
                qlen[g] = static_cast<int64_t>(q[g].size());
            const hough::serve::Choice ch = hough::serve::choose(
                n_grids, qlen.data(), pending_hits.data(), [&](int g, int64_t i) { return q[g][i].hits; },
                [&](int g, int64_t i) { return q[g][i].t; }, lanes.data(), static_cast<int>(lanes.size()), now,
                deadline, stop);
            wake = ch.wake;
            if (ch.lane < 0)
                break;
            int64_t hits = 0;
            std::printf("launch %.9f %d %d", now, ch.lane, ch.grid);
            for (int32_t k = 0; k < ch.take; ++k) {
                const Ev e = q[ch.grid].front();
                q[ch.grid].pop_front();
                pending_hits[ch.grid] -= e.hits;
                --n_pending;
                hits += e.hits;
                std::printf(" %d", e.id);
            }
            std::printf("\n");
            lanes[ch.lane].busy = true;
            busy_until[ch.lane] = now + svc_a + svc_b * static_cast<double>(hits);
        }
        double t_next = INFINITY;
        if (next < arrivals.size())
            t_next = std::min(t_next, arrivals[next].t);
        for (size_t k = 0; k < lanes.size(); ++k)
            if (lanes[k].busy)
                t_next = std::min(t_next, busy_until[k]);
        if (wake >= 0)
            t_next = std::min(t_next, wake > now ? wake : std::nextafter(now, INFINITY));
        if (!stop && stop_at > now)
            t_next = std::min(t_next, stop_at);
        if (!std::isfinite(t_next)) {
            if (n_pending == 0) {
                std::printf("end %.9f\n", now);
                return 0;
            }
            std::printf("stuck %.9f\n", now);
            return 1;
        }
        now = t_next;
    }
    std::printf("stuck %.9f\n", now);
    return 1;
}
