// Dispatch policy of the served stream (the server's rules in plain C++, with
// no HIP, so that a host program can drive them with a simulated clock and a
// fake executor).
//
// Events of one grid wait in arrival order.  A lane of that grid that is free
// takes the waiting events at once when no other lane of the grid is busy (an
// idle grid adds no latency).  While another lane of the grid is busy, the
// free lane waits to fill its batch until one of:
//   * the oldest waiting event has waited deadline_s;
//   * the waiting hits fill half of the lane's hit pool;
//   * the waiting events fill the lane's event slots;
//   * the server is stopping (everything left goes out).
// It then admits events from the front while the batch has a free event slot
// and room in the lane's hit pool, so a batch never reorders a grid's events.
// At submit, an event that no lane of its grid can ever hold is refused as
// invalid, and a full pending queue refuses it as busy.
#pragma once

#include <cstdint>

namespace hough {
namespace serve {

struct LaneState {
    int32_t grid;
    bool busy;
    int32_t max_events;   // event slots of a batch
    int64_t max_hits;     // hit pool of a batch
};

enum class Admit { ok, never_fits, queue_full };

inline Admit admit(int64_t n_hits, int64_t lane_pool, bool u16, int64_t n_pending, int64_t queue_limit) {
    if (n_hits > lane_pool || (u16 && n_hits > 65535))
        return Admit::never_fits;
    if (n_pending >= queue_limit)
        return Admit::queue_full;
    return Admit::ok;
}

struct Choice {
    int lane = -1;        // lane to launch now, or -1
    int grid = -1;
    int32_t take = 0;     // events taken from the front of that grid's queue
    double wake = -1.0;   // no launch: the earliest deadline still ahead, or -1 (wait for news)
};

// One decision over n_grids queues: queue_len[g] events wait for grid g,
// holding pending_hits[g] hits in all; hits_at(g, i) and submit_at(g, i) give
// the hit count and the submit time of the i-th waiting event of grid g
// (front first).  Grids are tried in order; the first lane that may launch is
// chosen.
template <typename HitsAt, typename SubmitAt>
Choice choose(int n_grids, const int64_t *queue_len, const int64_t *pending_hits, HitsAt hits_at,
              SubmitAt submit_at, const LaneState *lanes, int n_lanes, double now, double deadline_s, bool stop) {
    Choice c;
    for (int g = 0; g < n_grids; ++g) {
        if (queue_len[g] == 0)
            continue;
        int free_lane = -1;
        bool any_busy = false;
        for (int k = 0; k < n_lanes; ++k) {
            if (lanes[k].grid != g)
                continue;
            if (lanes[k].busy)
                any_busy = true;
            else if (free_lane < 0)
                free_lane = k;
        }
        if (free_lane < 0)
            continue;
        const LaneState &fl = lanes[free_lane];
        const double first = submit_at(g, 0);
        const bool go = !any_busy || stop || now - first >= deadline_s || 2 * pending_hits[g] >= fl.max_hits ||
                        queue_len[g] >= fl.max_events;
        if (!go) {
            const double at = first + deadline_s;
            c.wake = c.wake < 0 ? at : (at < c.wake ? at : c.wake);
            continue;
        }
        int64_t hits = 0;
        int32_t take = 0;
        while (take < queue_len[g] && take < fl.max_events && hits + hits_at(g, take) <= fl.max_hits) {
            hits += hits_at(g, take);
            ++take;
        }
        c.lane = free_lane;
        c.grid = g;
        c.take = take;
        c.wake = -1.0;
        return c;
    }
    return c;
}

}  // namespace serve
}  // namespace hough
