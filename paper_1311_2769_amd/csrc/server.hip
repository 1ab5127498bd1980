// Served trigger stream: one process drives the device as a trigger-farm node.
//
// Events of different sizes arrive one at a time (Section 1 and 2: the
// trigger sees a continuous stream of collisions; Section 4: events are
// independent).  The server keeps, per grid and per lane, a context, a stream
// and device-resident hit and candidate pools, and batches continuously: the
// moment a lane is free, the events waiting for its grid go out together as
// one hough_event_batch call, while the batches of the other lanes run.  An
// event waits for a batch slot, not for a fixed batch size:
//
//   * admission: an event fits a batch while the batch has a free event slot
//     (each slot owns one accumulator's worth of context workspace) and room
//     in the lane's hit pool; an event that can never fit is refused at
//     submit, and a full pending queue refuses with HOUGH_EBUSY;
//   * dispatch: a free lane takes its grid's waiting events at once when no
//     other lane of that grid is busy; otherwise it waits until the oldest
//     has waited `deadline_ms` or the waiting hits fill half a pool, so small
//     batches do not starve large ones;
//   * lanes: one worker thread per lane stages its batch's hits in pinned
//     memory, launches it, waits for it, copies each event's candidates
//     (exactly n_found of them) to the host and publishes the results with
//     their submit, launch and completion times; the dispatcher thread only
//     picks batches.
//
// The worker marks its phases as roctx ranges, so a rocprofv3 run with
// --marker-trace shows staging, waiting and the copy back per lane.
//
// Every result is the one hough_vote + hough_peaks give for that event alone:
// batching never changes an integer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dispatch.h"
#include "hough.h"
#include "hough_impl.h"

using namespace hough;

namespace {

using Clock = std::chrono::steady_clock;

struct Event {
    int64_t tag = 0;
    int32_t grid = 0;
    std::vector<float> x, y;
    double t_submit = 0.0;
};

struct Result {
    hough_served info{};
    std::vector<hough_cand> cands;
};

struct Lane {
    int32_t grid = 0;
    hough_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t max_events = 0;
    int64_t max_hits = 0;
    int64_t cap = 0;                 // candidate capacity per event
    float *x_d = nullptr, *y_d = nullptr;
    hough_cand *c_d = nullptr;
    int64_t *start_d = nullptr;      // packed list offsets of the batch in flight
    int32_t *nf_d = nullptr;
    uint64_t *nv_d = nullptr;
    float *x_h = nullptr, *y_h = nullptr;     // pinned
    hough_cand *c_h = nullptr;
    int32_t *nf_h = nullptr;
    uint64_t *nv_h = nullptr;
    // the batch in flight (filled by the dispatcher, then owned by the lane's worker)
    std::vector<std::unique_ptr<Event>> batch;
    std::vector<int64_t> hit_off, cand_off;
    double t_launch = 0.0;
    bool busy = false;               // guarded by the server mutex
    bool handed = false;             // a batch waits for the lane's worker
    std::thread worker;
};

}  // namespace

struct hough_server {
    int device = 0;
    Clock::time_point t0;
    std::vector<hough_grid> grids;
    std::vector<int32_t> thresholds;
    double deadline_s = 0.002;
    int32_t queue_limit = 4096;
    bool keep_candidates = true;
    double wait_limit_s = 10.0;             // longest wait for a batch before it fails
    std::vector<std::unique_ptr<Lane>> lanes;

    std::mutex mu;
    std::condition_variable cv_dispatch;    // new events, a free lane, stop
    std::condition_variable cv_lane;        // a batch handed to a lane's worker
    std::condition_variable cv_done;        // results published
    std::vector<std::deque<std::unique_ptr<Event>>> pending;   // per grid, FIFO
    std::vector<int64_t> pending_hits;
    int64_t n_pending = 0;
    std::deque<Result> done;
    bool stop = false;
    bool dispatch_over = false;             // the dispatcher has handed out its last batch
    std::thread dispatcher;
    std::string error;                      // first device failure, if any
    std::atomic<int64_t> refused{0};

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void set_error(hough_server *s, const char *what, hipError_t e) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error.empty())
        s->error = std::string(what) + ": " + hipGetErrorString(e);
}

// Bounded completion waits: poll the event (or stream) until it completes, a
// HIP error comes back, or limit_s seconds pass -- then an error, which
// fails the batch's events with HOUGH_EDEVICE instead of blocking the lane
// forever (hipErrorLaunchTimeOut stands for that limit).  Sleeps between
// polls grow from 10 us to 50 us, which bounds the delay a poll adds to an
// event's latency.
template <typename Query>
hipError_t wait_bounded(Query query, double limit_s) {
    const auto t_end = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double>(limit_s));
    auto nap = std::chrono::microseconds(10);
    while (true) {
        const hipError_t q = query();
        if (q != hipErrorNotReady)
            return q;
        if (Clock::now() >= t_end)
            return hipErrorLaunchTimeOut;   // reported as the batch time limit
        std::this_thread::sleep_for(nap);
        nap = std::min(nap * 2, std::chrono::microseconds(50));
    }
}

hipError_t wait_event(hipEvent_t ev, double limit_s) {
    return wait_bounded([&] { return hipEventQuery(ev); }, limit_s);
}

hipError_t wait_stream(hipStream_t st, double limit_s) {
    return wait_bounded([&] { return hipStreamQuery(st); }, limit_s);
}

template <typename T>
hipError_t dmalloc(T **p, size_t n) {
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T));
}

template <typename T>
hipError_t hmalloc(T **p, size_t n) {
    return hipHostMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault);
}

void free_lane(Lane *l) {
    if (l->ctx)
        hough_ctx_destroy(l->ctx);
    for (void *p : {static_cast<void *>(l->x_d), static_cast<void *>(l->y_d), static_cast<void *>(l->c_d),
                    static_cast<void *>(l->start_d), static_cast<void *>(l->nf_d), static_cast<void *>(l->nv_d)})
        if (p)
            (void)hipFree(p);
    for (void *p : {static_cast<void *>(l->x_h), static_cast<void *>(l->y_h), static_cast<void *>(l->c_h),
                    static_cast<void *>(l->nf_h), static_cast<void *>(l->nv_h)})
        if (p)
            (void)hipHostFree(p);
    if (l->done)
        (void)hipEventDestroy(l->done);
    if (l->stream)
        (void)hipStreamDestroy(l->stream);
}

// Candidate bound of one event of grid g (no two candidates are neighbours).
int64_t grid_bound(const hough_grid &g) {
    const int64_t a = (g.n_d0 + 1) / 2;
    const int64_t b = g.n_phi / 2;
    const int64_t c = (g.n_kappa + 1) / 2;
    return std::max<int64_t>(1, a * b * c);
}

// Stage and launch the lane's batch (the lane's worker, mutex not held): each
// lane copies its own events into pinned memory, so a large batch of one lane
// delays neither the dispatcher nor the other lanes.
hipError_t launch_batch(hough_server *s, Lane *l) {
    const int32_t n = static_cast<int32_t>(l->batch.size());
    l->hit_off.assign(n + 1, 0);
    l->cand_off.assign(n + 1, 0);
    for (int32_t e = 0; e < n; ++e) {
        const Event &ev = *l->batch[e];
        const int64_t h = l->hit_off[e];
        const size_t m = ev.x.size();
        std::memcpy(l->x_h + h, ev.x.data(), m * sizeof(float));
        std::memcpy(l->y_h + h, ev.y.data(), m * sizeof(float));
        l->hit_off[e + 1] = h + static_cast<int64_t>(m);
        l->cand_off[e + 1] = l->cand_off[e] + l->cap;
    }
    const int64_t hits = l->hit_off[n];
    hipError_t e = hipSuccess;
    if (hits > 0) {
        e = hipMemcpyAsync(l->x_d, l->x_h, hits * sizeof(float), hipMemcpyHostToDevice, l->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(l->y_d, l->y_h, hits * sizeof(float), hipMemcpyHostToDevice, l->stream);
    }
    if (e != hipSuccess)
        return e;
    l->t_launch = s->now();
    // packed lists: the completion thread copies a whole batch's candidates at once
    const hough_status st = hough_event_batch_packed(l->ctx, n, l->hit_off.data(), l->x_d, l->y_d,
                                                     s->thresholds[l->grid], nullptr, l->c_d, l->cand_off.data(),
                                                     l->start_d, l->nf_d, l->nv_d, l->stream);
    if (st != HOUGH_OK)
        return hipErrorLaunchFailure;
    e = hipMemcpyAsync(l->nf_h, l->nf_d, n * sizeof(int32_t), hipMemcpyDeviceToHost, l->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(l->nv_h, l->nv_d, n * sizeof(uint64_t), hipMemcpyDeviceToHost, l->stream);
    if (e == hipSuccess)
        e = hipEventRecord(l->done, l->stream);
    return e;
}

void dispatcher_main(hough_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    const int n_grids = static_cast<int>(s->grids.size());
    while (true) {
        if (s->stop && s->n_pending == 0) {
            // No batch will be handed out any more: completion threads may
            // leave once their lane is idle.
            s->dispatch_over = true;
            s->cv_lane.notify_all();
            break;
        }
        // the policy (dispatch.h) over the current queues and lanes
        std::vector<serve::LaneState> view(s->lanes.size());
        for (size_t k = 0; k < s->lanes.size(); ++k) {
            const Lane &l = *s->lanes[k];
            view[k] = serve::LaneState{l.grid, l.busy, l.max_events, l.max_hits};
        }
        std::vector<int64_t> qlen(static_cast<size_t>(n_grids));
        for (int g = 0; g < n_grids; ++g)
            qlen[g] = static_cast<int64_t>(s->pending[g].size());
        const serve::Choice ch = serve::choose(
            n_grids, qlen.data(), s->pending_hits.data(),
            [&](int g, int64_t i) { return static_cast<int64_t>(s->pending[g][i]->x.size()); },
            [&](int g, int64_t i) { return s->pending[g][i]->t_submit; }, view.data(),
            static_cast<int>(view.size()), s->now(), s->deadline_s, s->stop);
        const double wake = ch.wake;
        Lane *pick = nullptr;
        if (ch.lane >= 0) {
            pick = s->lanes[ch.lane].get();
            auto &q = s->pending[ch.grid];
            for (int32_t k = 0; k < ch.take; ++k) {
                s->pending_hits[ch.grid] -= static_cast<int64_t>(q.front()->x.size());
                pick->batch.push_back(std::move(q.front()));
                q.pop_front();
                --s->n_pending;
            }
            pick->busy = true;
        }
        if (!pick) {
            if (wake >= 0) {
                const double dt = std::max(0.0, wake - s->now());
                s->cv_dispatch.wait_for(lk, std::chrono::duration<double>(dt));
            } else {
                s->cv_dispatch.wait(lk);
            }
            continue;
        }
        pick->handed = true;
        s->cv_lane.notify_all();
    }
}

void lane_main(hough_server *s, Lane *l) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv_lane.wait(lk, [&] { return l->handed || (s->dispatch_over && !l->busy); });
        if (!l->handed)
            break;
        lk.unlock();
        const int32_t n = static_cast<int32_t>(l->batch.size());
        roctxRangePushA("hough_server: stage and launch a batch");
        hipError_t e = launch_batch(s, l);
        roctxRangePop();
        if (e != hipSuccess)
            set_error(s, "server batch launch", e);
        roctxRangePushA("hough_server: wait for a batch");
        if (e == hipSuccess)
            e = wait_event(l->done, s->wait_limit_s);
        roctxRangePop();
        roctxRangePushA("hough_server: candidates to the host");
        // The lists are packed: event k's min(n_found, cap) candidates follow
        // event k-1's, so one copy brings the whole batch's lists back.
        std::vector<int64_t> start(static_cast<size_t>(n) + 1, 0);
        for (int32_t k = 0; k < n && e == hipSuccess; ++k)
            start[k + 1] = start[k] + std::min<int64_t>(std::max(l->nf_h[k], 0), l->cap);
        if (e == hipSuccess && s->keep_candidates && start[n] > 0)
            e = hipMemcpyAsync(l->c_h, l->c_d, start[n] * sizeof(hough_cand), hipMemcpyDeviceToHost, l->stream);
        if (e == hipSuccess)
            e = wait_stream(l->stream, s->wait_limit_s);
        const double t_done = s->now();
        std::vector<Result> out(n);
        for (int32_t k = 0; k < n; ++k) {
            const Event &ev = *l->batch[k];
            Result &r = out[k];
            r.info.tag = ev.tag;
            r.info.grid = ev.grid;
            r.info.status = e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
            r.info.n_hits = static_cast<int32_t>(ev.x.size());
            r.info.n_found = e == hipSuccess ? l->nf_h[k] : 0;
            r.info.n_votes = e == hipSuccess ? l->nv_h[k] : 0;
            r.info.batch_events = n;
            r.info.t_submit = ev.t_submit;
            r.info.t_launch = l->t_launch;
            r.info.t_done = t_done;
            const int64_t m = (e == hipSuccess && s->keep_candidates) ? start[k + 1] - start[k] : 0;
            r.cands.assign(l->c_h + start[k], l->c_h + start[k] + m);
        }
        roctxRangePop();
        if (e != hipSuccess)
            set_error(s, "server batch completion", e);
        lk.lock();
        l->batch.clear();
        for (auto &r : out)
            s->done.push_back(std::move(r));
        l->handed = false;
        l->busy = false;
        s->cv_done.notify_all();
        s->cv_dispatch.notify_all();
    }
}

}  // namespace

extern "C" {

hough_status hough_server_create(hough_server **out, const hough_server_opts *o) {
    if (!out || !o || o->n_grids < 1 || o->n_grids > 8 || !o->grids || !o->thresholds)
        return HOUGH_EINVAL;
    *out = nullptr;
    const int lanes = o->lanes > 0 ? o->lanes : 2;
    if (lanes > 8 || o->deadline_ms < 0 || o->queue_limit < 0)
        return HOUGH_EINVAL;
    auto *s = new (std::nothrow) hough_server();
    if (!s)
        return HOUGH_ENOMEM;
    s->t0 = Clock::now();
    (void)hipGetDevice(&s->device);
    s->grids.assign(o->grids, o->grids + o->n_grids);
    s->thresholds.assign(o->thresholds, o->thresholds + o->n_grids);
    s->deadline_s = (o->deadline_ms > 0 ? o->deadline_ms : 2.0) * 1e-3;
    s->queue_limit = o->queue_limit > 0 ? o->queue_limit : 4096;
    s->keep_candidates = o->keep_candidates != 0;
    if (o->batch_timeout_ms < 0)
        return (delete s, HOUGH_EINVAL);
    s->wait_limit_s = (o->batch_timeout_ms > 0 ? o->batch_timeout_ms : 10000.0) * 1e-3;
    s->pending.resize(o->n_grids);
    s->pending_hits.assign(o->n_grids, 0);
    hough_status st = HOUGH_OK;
    hipError_t he = hipSuccess;
    for (int g = 0; g < o->n_grids && st == HOUGH_OK; ++g) {
        const hough_grid &grid = s->grids[g];
        const int32_t E = (o->batch_events && o->batch_events[g] > 0) ? o->batch_events[g] : 64;
        const int64_t H = (o->batch_hits && o->batch_hits[g] > 0) ? o->batch_hits[g] : (int64_t{1} << 22);
        const int64_t bound = grid_bound(grid);
        const int64_t cap = (o->event_candidates && o->event_candidates[g] > 0)
                                ? std::min(o->event_candidates[g], bound) : bound;
        for (int k = 0; k < lanes && st == HOUGH_OK; ++k) {
            auto l = std::make_unique<Lane>();
            l->grid = g;
            l->max_events = E;
            l->max_hits = H;
            l->cap = cap;
            hough_ctx_opts co{};
            co.max_events = E;
            co.max_hits = H;
            co.tune_cache = o->tune_cache;
            st = hough_ctx_create(&l->ctx, &grid, &co);
            if (st != HOUGH_OK) {
                s->lanes.push_back(std::move(l));
                break;
            }
            he = hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking);
            he = he ? he : hipEventCreateWithFlags(&l->done, hipEventDisableTiming | hipEventBlockingSync);
            he = he ? he : dmalloc(&l->x_d, H);
            he = he ? he : dmalloc(&l->y_d, H);
            he = he ? he : dmalloc(&l->c_d, static_cast<size_t>(E) * cap);
            he = he ? he : dmalloc(&l->start_d, static_cast<size_t>(E) + 1);
            he = he ? he : dmalloc(&l->nf_d, E);
            he = he ? he : dmalloc(&l->nv_d, E);
            he = he ? he : hmalloc(&l->x_h, H);
            he = he ? he : hmalloc(&l->y_h, H);
            he = he ? he : hmalloc(&l->c_h, static_cast<size_t>(E) * cap);
            he = he ? he : hmalloc(&l->nf_h, E);
            he = he ? he : hmalloc(&l->nv_h, E);
            if (he != hipSuccess)
                st = (he == hipErrorOutOfMemory || he == hipErrorMemoryAllocation) ? HOUGH_ENOMEM : HOUGH_EDEVICE;
            s->lanes.push_back(std::move(l));
        }
    }
    if (st != HOUGH_OK) {
        for (auto &l : s->lanes)
            free_lane(l.get());
        delete s;
        return st;
    }
    for (auto &l : s->lanes)
        l->worker = std::thread(lane_main, s, l.get());
    s->dispatcher = std::thread(dispatcher_main, s);
    *out = s;
    return HOUGH_OK;
}

void hough_server_destroy(hough_server *s) {
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_dispatch.notify_all();
    if (s->dispatcher.joinable())
        s->dispatcher.join();           // launches everything still pending
    {
        std::lock_guard<std::mutex> lk(s->mu);
    }
    s->cv_lane.notify_all();
    for (auto &l : s->lanes)
        if (l->worker.joinable())
            l->worker.join();
    for (auto &l : s->lanes)
        free_lane(l.get());
    delete s;
}

double hough_server_clock(const hough_server *s) { return s ? s->now() : 0.0; }

hough_status hough_server_submit(hough_server *s, int64_t tag, int32_t grid, const float *x, const float *y,
                                 int32_t n_hits, double t_submit) {
    if (!s || grid < 0 || grid >= static_cast<int32_t>(s->grids.size()) || n_hits < 0 ||
        (n_hits > 0 && (!x || !y)))
        return HOUGH_EINVAL;
    int64_t pool = 0;
    for (auto &l : s->lanes)
        if (l->grid == grid)
            pool = l->max_hits;
    const bool u16 = s->grids[grid].acc_type == HOUGH_ACC_U16;
    if (serve::admit(n_hits, pool, u16, 0, 1) == serve::Admit::never_fits)
        return HOUGH_EINVAL;         // can never be admitted
    auto ev = std::make_unique<Event>();
    ev->tag = tag;
    ev->grid = grid;
    ev->x.assign(x, x + n_hits);
    ev->y.assign(y, y + n_hits);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop)
            return HOUGH_EINVAL;
        if (serve::admit(n_hits, pool, u16, s->n_pending, s->queue_limit) == serve::Admit::queue_full) {
            ++s->refused;
            return HOUGH_EBUSY;
        }
        ev->t_submit = t_submit >= 0 ? t_submit : s->now();
        s->pending_hits[grid] += n_hits;
        s->pending[grid].push_back(std::move(ev));
        ++s->n_pending;
    }
    s->cv_dispatch.notify_one();
    return HOUGH_OK;
}

hough_status hough_server_replay(hough_server *s, int32_t n, const double *arrival_s, const int32_t *pick,
                                 int32_t n_pool, const int32_t *pool_grid, const int64_t *pool_hit_off,
                                 const float *pool_x, const float *pool_y, int32_t *status) {
    if (!s || n < 0 || n_pool < 0 || (n > 0 && (!arrival_s || !pick || !status || n_pool == 0)) ||
        (n_pool > 0 && (!pool_grid || !pool_hit_off)))
        return HOUGH_EINVAL;
    for (int32_t k = 0; k < n_pool; ++k)
        if (pool_hit_off[k + 1] < pool_hit_off[k])
            return HOUGH_EINVAL;
    for (int32_t i = 0; i < n; ++i)
        if (pick[i] < 0 || pick[i] >= n_pool || (i > 0 && arrival_s[i] < arrival_s[i - 1]))
            return HOUGH_EINVAL;
    const double base = s->now();
    for (int32_t i = 0; i < n; ++i) {
        const double due = base + arrival_s[i];
        // sleep to within 100 us of the arrival, then spin
        for (double left = due - s->now(); left > 0; left = due - s->now()) {
            if (left > 2e-4)
                std::this_thread::sleep_for(std::chrono::duration<double>(left - 1e-4));
        }
        const int32_t k = pick[i];
        const int64_t a = pool_hit_off[k];
        status[i] = hough_server_submit(s, i, pool_grid[k], pool_x + a, pool_y + a,
                                        static_cast<int32_t>(pool_hit_off[k + 1] - a), due);
    }
    return HOUGH_OK;
}

hough_status hough_server_poll(hough_server *s, hough_served *out, int32_t max_out, hough_cand *cand_buf,
                               int64_t cand_cap, int32_t *n_out, int32_t wait_ms) {
    if (!s || !n_out || max_out < 0 || (max_out > 0 && !out) || cand_cap < 0 || (cand_cap > 0 && !cand_buf))
        return HOUGH_EINVAL;
    *n_out = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int64_t used = 0;
    int32_t k = 0;
    while (k < max_out && !s->done.empty()) {
        Result &r = s->done.front();
        const int64_t m = static_cast<int64_t>(r.cands.size());
        if (used + m > cand_cap && k > 0)
            break;                                   // the rest goes to the next poll
        const int64_t stored = std::min(m, cand_cap - used);
        if (stored > 0)
            std::memcpy(cand_buf + used, r.cands.data(), stored * sizeof(hough_cand));
        out[k] = r.info;
        out[k].cand_offset = used;
        out[k].n_stored = static_cast<int32_t>(stored);
        used += stored;
        ++k;
        s->done.pop_front();
    }
    *n_out = k;
    if (!s->error.empty()) {
        ::set_last_error(s->error.c_str());
        return HOUGH_EDEVICE;
    }
    return HOUGH_OK;
}

hough_status hough_server_stats(hough_server *s, int64_t *pending, int64_t *refused, int32_t *busy_lanes) {
    if (!s)
        return HOUGH_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (pending)
        *pending = s->n_pending;
    if (refused)
        *refused = s->refused.load();
    if (busy_lanes) {
        int32_t b = 0;
        for (auto &l : s->lanes)
            b += l->busy ? 1 : 0;
        *busy_lanes = b;
    }
    return HOUGH_OK;
}

}  // extern "C"
