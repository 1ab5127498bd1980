// C ABI of libhough: contexts, argument checking, workspace and launch
// sequences.  See include/hough.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "hough.h"
#include "hough_impl.h"
#include "assoc.h"

using namespace hough;

namespace {

thread_local std::string g_last_error;

hough_status device_error(hipError_t e, const char *what) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
    g_last_error = buf;
    return HOUGH_EDEVICE;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess)                           \
            return device_error(e_, #expr);             \
    } while (0)

// Descriptor block uploaded per batch: a header followed by per-event
// descriptors and the work list.
struct BatchHeader {
    int32_t n_events;
    int32_t n_items;
    int64_t n_hits;
    QueueDesc queues;
};

struct GraphKey {
    const void *x, *y, *acc, *cands, *n_found, *n_votes, *cand_start;
    int32_t threshold;
    int64_t hit_bucket;
    uint32_t key_mask;      // sort-key digits that can differ (sets the sort passes)
    bool operator==(const GraphKey &o) const {
        return x == o.x && y == o.y && acc == o.acc && cands == o.cands && n_found == o.n_found &&
               n_votes == o.n_votes && cand_start == o.cand_start && threshold == o.threshold && hit_bucket == o.hit_bucket &&
               key_mask == o.key_mask;
    }
};

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
};

// Tile heights a batched vote can use; workspace is sized for all of them.
constexpr int32_t kBatchRows[] = {32, 64, 128};

}  // namespace

struct hough_ctx {
    hough_grid grid;
    GridArgs g;
    bool u16;
    bool fused_batch;          // 2D int32: peaks searched inside the vote tiles
    bool cull_ok;              // phi0 table holds the bin centres (n_phi <= 32768): arcs allowed
    int32_t max_events;
    int64_t max_hits;
    int device;
    VoteShape shape_single;
    VoteShape shape_batch;
    int32_t cus;                  // compute units of the device (persistent launches)

    // sort workspace
    int64_t bound;             // max candidates per event (any first-pass layout)
    int32_t hist_chunks;
    int32_t max_blocks0;
    EventState *state = nullptr;
    Cand *stage = nullptr;     // also the second ping-pong buffer
    int32_t *cnt0 = nullptr;
    uint32_t *hist = nullptr;
    Cand *tmp0 = nullptr;
    uint32_t *acc_ws = nullptr;   // batch accumulators when the caller passes none
    float4 *hits = nullptr;       // [max_hits] hit records written by hit_prep
    uint2 *ranges = nullptr;      // [n_d0][max_hits] tile ranges per hit, when cull_ok
    uint2 *all_tiles = nullptr;   // one all-tiles entry: culling off
    int32_t *cell_map = nullptr;  // [cells] hit association: 1 + candidate index per cell
    uint32_t *cell_bits = nullptr;  // hit association: bitmap of the cells that hold a candidate
    int32_t *assoc_hist = nullptr;  // hit association: azimuth bucket counts and offsets

    // batch descriptors
    size_t desc_bytes = 0;
    char *desc_host = nullptr;    // pinned
    char *desc_dev = nullptr;
    int32_t *work_counter = nullptr;
    int32_t max_items = 0;
    hipEvent_t desc_done = nullptr;
    bool desc_in_flight = false;
    std::vector<int64_t> last_hit_off, last_cand_off;   // what desc_host currently holds
    bool last_fused = false;                             // ... and for which tile layout
    hipStream_t capture_stream = nullptr;
    std::vector<GraphEntry> graphs;

    // timing mode: batches run without a graph, with events around the vote
    bool timing = false;
    bool count_pairs = false;  // timing mode 2: the vote also counts the pairs it evaluates
    bool timed_once = false;
    unsigned long long *pairs = nullptr;   // timing mode: (hit, row) pairs the last timed vote evaluated
    hipEvent_t ev_start = nullptr, ev_vote0 = nullptr, ev_vote1 = nullptr, ev_end = nullptr;
};

namespace {

void drop_graphs(hough_ctx *c) {
    for (auto &ge : c->graphs)
        (void)hipGraphExecDestroy(ge.exec);
    c->graphs.clear();
}

void free_ctx(hough_ctx *c) {
    if (!c)
        return;
    drop_graphs(c);
    for (hipEvent_t ev : {c->desc_done, c->ev_start, c->ev_vote0, c->ev_vote1, c->ev_end})
        if (ev)
            (void)hipEventDestroy(ev);
    if (c->capture_stream)
        (void)hipStreamDestroy(c->capture_stream);
    if (c->desc_host)
        (void)hipHostFree(c->desc_host);
    void *dev[] = {c->state, c->stage, c->cnt0, c->hist, c->tmp0, c->acc_ws, c->hits, c->ranges, c->all_tiles,
                   c->desc_dev, c->work_counter, c->cell_map, c->cell_bits, c->pairs, c->assoc_hist};
    for (void *p : dev)
        if (p)
            (void)hipFree(p);
    delete c;
}

int32_t batch_tiles_per_event(const hough_ctx *c, const VoteShape &s, bool fused) {
    return vote_slice_units(c->g, c->u16) * vote_tiles_per_slice(c->g, s, fused);
}

// Tile words instead of ranges when culling is on and a slice has few enough tiles.
bool use_masks(const hough_ctx *c, const VoteShape &s, bool fused) {
    return c->cull_ok && vote_tile_geom(c->g, s, fused).tiles <= kMaskTiles;
}

VoteInputs vote_inputs(const hough_ctx *c, const VoteShape &s, bool fused) {
    VoteInputs in{};
    in.hits = c->hits;
    in.ranges = c->cull_ok ? c->ranges : c->all_tiles;
    in.mask_mode = use_masks(c, s, fused) ? 1 : 0;
    in.range_stride = !c->cull_ok ? 0 : in.mask_mode ? tile_word_stride(c->max_hits) : c->max_hits;
    in.range_step = c->cull_ok ? 1 : 0;
    return in;
}

// Hit records (and tile ranges or words) for a vote launch of shape s.
hipError_t hit_prep(const hough_ctx *c, const VoteShape &s, bool fused, const float *x, const float *y,
                    int64_t n_hits, const int64_t *n_hits_dev, hipStream_t stream) {
    const bool words = use_masks(c, s, fused);
    return launch_hit_prep(c->g, vote_tile_geom(c->g, s, fused), x, y, n_hits, n_hits_dev, c->hits,
                           c->cull_ok ? c->ranges : nullptr, words ? tile_word_stride(c->max_hits) : c->max_hits,
                           c->cull_ok, words, nullptr, stream);
}

SortWork sort_work(const hough_ctx *c, bool fused_layout) {
    SortWork w{};
    w.s0.stage = c->stage;
    w.s0.cnt0 = c->cnt0;
    if (fused_layout) {
        w.s0.n_blocks0 = vote_tiles_per_slice(c->g, c->shape_batch, true);
        w.s0.cap0 = fused_chunk_cap(c->g, c->shape_batch);
        w.s0.cb = 1;
    } else {
        w.s0.n_blocks0 = peak_blocks_per_event(c->g);
        w.s0.cap0 = peak_block_cap(c->g);
        w.s0.cb = peak_blocks_per_chunk(c->g);
    }
    w.hist = c->hist;
    w.hist_chunks = c->hist_chunks;
    w.tmp0 = c->tmp0;
    w.tmp1 = c->stage;
    w.bound = c->bound;
    w.state = c->state;
    w.key_mask = c->u16 ? 0xffffu : 0xffffffffu;
    return w;
}

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    if (count == 0)
        count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

// Does the phi0 table hold the bin centres (j + 1/2) 2 pi / n_phi?  The tile
// masks assume it; any other table just turns culling off.
bool table_is_bin_centres(const hough_grid *grid) {
    const size_t n = static_cast<size_t>(grid->n_phi);
    std::vector<float> c(n), s(n);
    if (hipMemcpy(c.data(), grid->cos_phi, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(s.data(), grid->sin_phi, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return false;
    const double two_pi = 6.283185307179586;
    for (size_t j = 0; j < n; ++j) {
        const double want = (static_cast<double>(j) + 0.5) * two_pi / static_cast<double>(n);
        const double got = std::atan2(static_cast<double>(s[j]), static_cast<double>(c[j]));
        double diff = std::fmod(got - want, two_pi);
        if (diff > two_pi / 2)
            diff -= two_pi;
        if (diff < -two_pi / 2)
            diff += two_pi;
        const double norm = std::hypot(static_cast<double>(c[j]), static_cast<double>(s[j]));
        if (!(std::fabs(diff) < 1e-6) || !(std::fabs(norm - 1.0) < 1e-6))
            return false;
    }
    return true;
}

// Write the batch descriptors (header, per-event ranges, largest-first work
// list) into the pinned staging block, unless it already holds this batch.
// *changed tells the caller whether the device copy must be refreshed.
hough_status stage_descriptors(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off,
                               const int64_t *cand_off, bool fused, bool *changed) {
    const size_t n = static_cast<size_t>(n_events) + 1;
    std::vector<int64_t> co(n, 0);
    if (cand_off)
        co.assign(cand_off, cand_off + n);
    if (ctx->last_hit_off.size() == n && std::equal(hit_off, hit_off + n, ctx->last_hit_off.begin()) &&
        ctx->last_cand_off == co && ctx->last_fused == fused) {
        *changed = false;
        return HOUGH_OK;
    }
    // The previous upload must have left the pinned block before it is rewritten.
    if (ctx->desc_in_flight)
        HIP_TRY(hipEventSynchronize(ctx->desc_done));
    ctx->desc_in_flight = false;
    const int32_t tpe = batch_tiles_per_event(ctx, ctx->shape_batch, fused);
    auto *hdr = reinterpret_cast<BatchHeader *>(ctx->desc_host);
    auto *desc = reinterpret_cast<EventDesc *>(ctx->desc_host + sizeof(BatchHeader));
    auto *items = reinterpret_cast<WorkItem *>(ctx->desc_host + sizeof(BatchHeader) +
                                               static_cast<size_t>(ctx->max_events) * sizeof(EventDesc));
    hdr->n_events = n_events;
    hdr->n_items = n_events * tpe;
    hdr->n_hits = hit_off[n_events];
    for (int32_t e = 0; e < n_events; ++e) {
        desc[e].hit_begin = hit_off[e];
        desc[e].hit_end = hit_off[e + 1];
        desc[e].cand_begin = co[e];
        desc[e].cand_cap = static_cast<int32_t>(co[e + 1] - co[e]);
        desc[e].pad_ = 0;
    }
    // Events go whole to the XCD queues, largest first, each to the queue with
    // the least work so far (a tile's work grows with the event's hits, plus
    // a fixed part for its clear and peak scan), so the queues drain together
    // and every tile of an event reads its hits through one L2.
    std::vector<int32_t> order(static_cast<size_t>(n_events));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return hit_off[a + 1] - hit_off[a] > hit_off[b + 1] - hit_off[b];
    });
    std::vector<int32_t> queue_of(static_cast<size_t>(n_events));
    int64_t load[kQueues] = {};
    for (int32_t e : order) {
        const int q = static_cast<int>(std::min_element(load, load + kQueues) - load);
        queue_of[e] = q;
        load[q] += (hit_off[e + 1] - hit_off[e] + 1024) * tpe;
    }
    int32_t n_items = 0;
    for (int q = 0; q < kQueues; ++q) {
        hdr->queues.begin[q] = n_items;
        for (int32_t e : order)
            if (queue_of[e] == q)
                for (int32_t t = 0; t < tpe; ++t)
                    items[n_items++] = WorkItem{e, t};
        hdr->queues.len[q] = n_items - hdr->queues.begin[q];
    }
    ctx->last_hit_off.assign(hit_off, hit_off + n);
    ctx->last_cand_off = co;
    ctx->last_fused = fused;
    *changed = true;
    return HOUGH_OK;
}

hough_status check_batch(const hough_ctx *ctx, int32_t n_events, const int64_t *hit_off, const float *x,
                         const float *y) {
    if (!ctx || !hit_off || n_events < 1 || n_events > ctx->max_events || hit_off[0] != 0)
        return HOUGH_EINVAL;
    for (int32_t e = 0; e < n_events; ++e) {
        const int64_t nh = hit_off[e + 1] - hit_off[e];
        if (nh < 0 || (ctx->u16 && nh > 65535))
            return HOUGH_EINVAL;
    }
    if (hit_off[n_events] > ctx->max_hits)
        return HOUGH_EINVAL;
    if (hit_off[n_events] > 0 && (!x || !y))
        return HOUGH_EINVAL;
    return HOUGH_OK;
}

struct DevDesc {
    BatchHeader *hdr;
    EventDesc *desc;
    WorkItem *items;
};

DevDesc device_descriptors(const hough_ctx *ctx) {
    char *dd = ctx->desc_dev;
    DevDesc d;
    d.hdr = reinterpret_cast<BatchHeader *>(dd);
    d.desc = reinterpret_cast<EventDesc *>(dd + sizeof(BatchHeader));
    d.items = reinterpret_cast<WorkItem *>(dd + sizeof(BatchHeader) +
                                           static_cast<size_t>(ctx->max_events) * sizeof(EventDesc));
    return d;
}

// Hit counts are rounded up to a power of two (at least kHitBucket) in the
// captured graphs -- the exact count is read on the device -- so a context
// needs at most a few graphs whatever its batches hold.
constexpr int64_t kHitBucket = 1 << 16;
constexpr size_t kMaxGraphs = 32;         // executable graphs kept per context

// Sort-key digits that can differ within the events of a batch.  A key is
// 0x7fffffff - votes, which is 0x7fffffff XOR votes for 0 <= votes, so two
// keys differ only within the bits of the larger count.  A cell takes at most
// one vote per hit (one kappa bin per (d0, phi0) row), so an event of n hits
// has counts of at most n, and uint16 cells at most 65535.
uint32_t batch_key_mask(const hough_ctx *ctx, int32_t n_events, const int64_t *hit_off) {
    int64_t most = 0;
    for (int32_t e = 0; e < n_events; ++e)
        most = std::max(most, hit_off[e + 1] - hit_off[e]);
    if (ctx->u16)
        most = std::min<int64_t>(most, 0xffff);
    uint32_t mask = 0;
    while (mask < 0x7fffffffu && static_cast<int64_t>(mask) < most)
        mask = (mask << 1) | 1u;
    return mask;
}

int64_t hit_bucket(int64_t hits) {
    int64_t b = kHitBucket;
    while (b < hits)
        b <<= 1;
    return b;
}


// The launch sequence of one batch (after the descriptor upload): reset,
// tile words, vote (fused with the peak search for 2D int32), sort.  With
// `timed`, events bracket the whole sequence and the vote kernel.
hipError_t enqueue_batch(hough_ctx *ctx, hipStream_t cs, const float *x, const float *y, int32_t threshold,
                         void *acc, hough_cand *cands, int32_t *n_found, uint64_t *n_votes, int64_t *cand_start,
                         int64_t bucket, uint32_t key_mask, bool timed) {
    DevDesc dd = device_descriptors(ctx);
    const VoteShape &vs = ctx->shape_batch;
    const bool fused = ctx->fused_batch;
    SortWork w = sort_work(ctx, fused);
    w.key_mask = key_mask;
    w.desc = dd.desc;
    w.out = cands;
    w.n_found = n_found;
    w.n_events_dev = &dd.hdr->n_events;
    w.cand_start = cand_start;
    auto *nv = reinterpret_cast<unsigned long long *>(n_votes);
    uint32_t *acc_dw = static_cast<uint32_t *>(acc);
    hipError_t ce = hipSuccess;
    if (timed)
        ce = hipEventRecord(ctx->ev_start, cs);
    if (ce == hipSuccess)
        ce = launch_prep_batch(ctx->state, ctx->max_events, &dd.hdr->n_events, nv, ctx->work_counter, cs);
    if (ce == hipSuccess)
        ce = hit_prep(ctx, vs, fused, x, y, bucket, &dd.hdr->n_hits, cs);
    if (ce == hipSuccess && timed)
        ce = hipEventRecord(ctx->ev_vote0, cs);
    uint32_t *a = (fused || acc_dw) ? acc_dw : ctx->acc_ws;
    const bool count = timed && ctx->count_pairs;
    if (ce == hipSuccess && count)
        ce = launch_zero(reinterpret_cast<uint32_t *>(ctx->pairs), 2, cs);
    if (ce == hipSuccess)
        ce = launch_vote_batch(ctx->g, ctx->u16, fused, vs, vote_inputs(ctx, vs, fused), dd.desc,
                               &dd.hdr->queues, dd.items, ctx->max_items, ctx->work_counter,
                               ctx->cus * vote_groups_per_cu(vs, ctx->g.n_kappa), a, nv, fused ? &w : nullptr,
                               threshold, cs,
                               count ? ctx->pairs : nullptr);
    if (ce == hipSuccess && timed)
        ce = hipEventRecord(ctx->ev_vote1, cs);
    if (ce == hipSuccess && !fused)
        ce = launch_peaks(ctx->g, ctx->u16, a, ctx->max_events, threshold, w, cs);
    if (ce == hipSuccess)
        ce = launch_sort(w, ctx->max_events, cs);
    if (ce == hipSuccess && timed)
        ce = hipEventRecord(ctx->ev_end, cs);
    return ce;
}

}  // namespace

void set_last_error(const char *msg) { g_last_error = msg ? msg : ""; }

namespace hough {

hough_status grid_setup(const hough_grid *grid, GridArgs *out) {
    if (!grid || !out)
        return HOUGH_EINVAL;
    if (grid->n_phi < 3 || grid->n_kappa < 1 || grid->n_d0 < 1 || !grid->cos_phi || !grid->sin_phi)
        return HOUGH_EINVAL;
    if (grid->n_d0 > 1 && !grid->d0)
        return HOUGH_EINVAL;
    if (grid->family != HOUGH_CURVED && grid->family != HOUGH_STRAIGHT)
        return HOUGH_EINVAL;
    if (grid->family == HOUGH_STRAIGHT && (grid->n_d0 != 1 || grid->d0 != nullptr))
        return HOUGH_EINVAL;
    if (grid->forward != 0 && grid->forward != 1)
        return HOUGH_EINVAL;
    if (grid->acc_type != HOUGH_ACC_I32 && grid->acc_type != HOUGH_ACC_U16)
        return HOUGH_EINVAL;
    const bool u16 = grid->acc_type == HOUGH_ACC_U16;
    if (u16 && (grid->n_kappa & 1))
        return HOUGH_EINVAL;
    const int64_t cells = static_cast<int64_t>(grid->n_d0) * grid->n_phi * grid->n_kappa;
    if (cells > 0x7fffffffLL)
        return HOUGH_EINVAL;
    GridArgs g{};
    g.cos_phi = grid->cos_phi;
    g.sin_phi = grid->sin_phi;
    g.d0 = grid->d0;
    g.n_d0 = grid->n_d0;
    g.n_phi = grid->n_phi;
    g.n_kappa = grid->n_kappa;
    // kappa_min = +0 is stored as -0: kf = (kappa - kappa_min) * kappa_scale
    // then differs only for kappa = -0, where it is +0 instead of -0 (both vote
    // bin 0), and is never -0 when kappa_scale >= 1 (see the vote's range test).
    g.kappa_min = (grid->kappa_min == 0.0f) ? -0.0f : grid->kappa_min;
    g.kappa_scale = grid->kappa_scale;
    g.bin_bits = grid->kappa_scale >= 1.0f ? 1 : 0;
    g.near_band = -1.0f;
    g.kf_off = 0.0f;
    g.kscale2 = 2.0f * grid->kappa_scale;
    g.straight = grid->family == HOUGH_STRAIGHT ? 1 : 0;
    g.forward = grid->forward;
    g.row_dwords = u16 ? grid->n_kappa / 2 : grid->n_kappa;
    g.cells = cells;
    g.acc_dwords = static_cast<int64_t>(grid->n_d0) * grid->n_phi * g.row_dwords;
    float band = 0.0f, off = 0.0f;
    if (vote_near_band(g, &band, &off)) {
        g.near_band = band;
        g.kf_off = off;
    }
    *out = g;
    return HOUGH_OK;
}

int32_t default_tile_rows(const GridArgs &g, bool u16) {
    // Slice pairs (uint16 with a d0 axis): 32 rows, three workgroups per CU
    // (the displaced batch votes 4 % faster than with 64).  Otherwise 64 rows
    // while two such workgroups still fit a CU's LDS (n_kappa <= 256: each hit
    // is staged half as often), else 32.  The forward kernels come in 32-row
    // tiles.
    if (u16 && g.d0)
        return 32;
    return (g.n_kappa <= 256 && g.forward == 0) ? 64 : 32;
}

}  // namespace hough

void ctx_grid(const hough_ctx *ctx, hough_grid *out) { *out = ctx->grid; }

extern "C" {

const char *hough_version(void) { return "hough-mi355x 0.2"; }

const char *hough_status_str(hough_status s) {
    switch (s) {
        case HOUGH_OK: return "ok";
        case HOUGH_EINVAL: return "invalid argument";
        case HOUGH_ENOMEM: return "out of device memory";
        case HOUGH_EDEVICE: return "HIP runtime error";
        case HOUGH_EBUSY: return "busy: the server's queue is full";
    }
    return "unknown status";
}

const char *hough_last_error(void) { return g_last_error.c_str(); }

hough_status hough_ctx_create(hough_ctx **out, const hough_grid *grid, const hough_ctx_opts *opts) {
    if (!out || !grid)
        return HOUGH_EINVAL;
    *out = nullptr;
    GridArgs ga{};
    if (grid_setup(grid, &ga) != HOUGH_OK)
        return HOUGH_EINVAL;
    const bool u16 = grid->acc_type == HOUGH_ACC_U16;
    hough_ctx_opts o{};
    if (opts)
        o = *opts;
    if (o.max_events < 0 || o.max_hits < 0)
        return HOUGH_EINVAL;
    if (o.max_events == 0)
        o.max_events = 1;
    if (o.max_hits == 0)
        o.max_hits = 1 << 20;
    if (o.max_hits > (int64_t{1} << 30))
        return HOUGH_EINVAL;     // the vote kernels index hit records with 32 bits

    hough_ctx *c = new (std::nothrow) hough_ctx();
    if (!c)
        return HOUGH_ENOMEM;
    c->grid = *grid;
    c->u16 = u16;
    c->max_events = o.max_events;
    c->max_hits = o.max_hits;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return device_error(hipErrorNoDevice, "hipGetDevice");
    }
    c->g = ga;
    const GridArgs &g = c->g;
    c->fused_batch = !u16 && grid->d0 == nullptr;

    // Default launch shapes (the autotuner may replace them).
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, c->device);
    const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    const int32_t rows = default_tile_rows(g, u16);
    c->shape_single = VoteShape{rows, 512, u16 ? 1 : 4};
    c->shape_batch = VoteShape{rows, 512, 1};
    if (!vote_shape_supported(c->shape_single, u16, g.n_kappa, g.forward != 0) ||
        !vote_shape_supported(c->shape_batch, u16, g.n_kappa, g.forward != 0)) {
        delete c;
        return HOUGH_EINVAL;   // a kappa row too long for an LDS tile
    }
    c->cus = cus;
    // Tuned shapes for this device, grid and size, if the cache has them.
    if (const char *cache = tune_cache_path(o.tune_cache)) {
        TuneEntry key;
        key.device = device_tag(c->device);
        key.n_d0 = grid->n_d0;
        key.n_phi = grid->n_phi;
        key.n_kappa = grid->n_kappa;
        key.acc = grid->acc_type;
        key.hits_log2 = tune_hits_log2(o.max_hits);
        for (int which = 0; which < 2; ++which) {
            key.which = which;
            TuneEntry e;
            if (!tune_lookup(cache, key, &e))
                continue;
            const VoteShape s{e.rows, e.threads, which == 1 ? 1 : e.split};
            if (vote_shape_supported(s, u16, g.n_kappa, g.forward != 0))
                (which == 0 ? c->shape_single : c->shape_batch) = s;
        }
    }
    c->cull_ok = grid->n_phi <= 32768 && table_is_bin_centres(grid);

    // Sort workspace sized for every first-pass layout: peak blocks, and
    // fused tiles of each batched tile height.
    const int32_t pb = peak_blocks_per_event(g);
    int64_t bound = static_cast<int64_t>(pb) * peak_block_cap(g);
    int32_t first_chunks = (pb + peak_blocks_per_chunk(g) - 1) / peak_blocks_per_chunk(g);
    int32_t max_blocks = pb;
    if (c->fused_batch) {
        for (int32_t rows : kBatchRows) {
            VoteShape s{rows, 256, 1};
            const int32_t tiles = vote_tiles_per_slice(g, s, true);
            bound = std::max<int64_t>(bound, static_cast<int64_t>(tiles) * fused_chunk_cap(g, s));
            first_chunks = std::max(first_chunks, tiles);
            max_blocks = std::max(max_blocks, tiles);
        }
    }
    c->bound = bound;
    c->max_blocks0 = max_blocks;
    const int64_t later = (c->bound + kSortChunk - 1) / kSortChunk;
    c->hist_chunks = static_cast<int32_t>(std::max<int64_t>(first_chunks, later));
    const size_t E = static_cast<size_t>(c->max_events);
    int32_t max_tpe = 0;
    for (int32_t rows : kBatchRows)
        max_tpe = std::max(max_tpe, vote_slice_units(g, c->u16) *
                                        vote_tiles_per_slice(g, VoteShape{rows, 256, 1}, c->fused_batch));
    c->max_items = static_cast<int32_t>(E) * max_tpe;
    c->desc_bytes = sizeof(BatchHeader) + E * sizeof(EventDesc) + static_cast<size_t>(c->max_items) * sizeof(WorkItem);

    hipError_t e = hipSuccess;
    e = e ? e : dev_alloc(&c->state, E);
    e = e ? e : dev_alloc(&c->stage, E * static_cast<size_t>(c->bound));
    e = e ? e : dev_alloc(&c->cnt0, E * static_cast<size_t>(c->max_blocks0));
    e = e ? e : dev_alloc(&c->hist, E * static_cast<size_t>(c->hist_chunks) * kDigits);
    e = e ? e : dev_alloc(&c->tmp0, E * static_cast<size_t>(c->bound));
    e = e ? e : dev_alloc(&c->acc_ws, E * static_cast<size_t>(g.acc_dwords));
    e = e ? e : dev_alloc(&c->hits, static_cast<size_t>(c->max_hits));
    if (c->cull_ok)
        e = e ? e : dev_alloc(&c->ranges, static_cast<size_t>(g.n_d0) * static_cast<size_t>(ranges_entries(c->max_hits)));
    e = e ? e : dev_alloc(&c->all_tiles, 1);
    e = e ? e : dev_alloc(&c->cell_map, static_cast<size_t>(g.cells));
    e = e ? e : dev_alloc(&c->cell_bits, static_cast<size_t>(g.n_d0) * static_cast<size_t>(g.n_phi) *
                                             static_cast<size_t>(assoc_row_words(g.n_kappa)));
    if (e == hipSuccess) {
        const uint2 all = make_uint2(kAllTiles, 0u);
        e = hipMemcpy(c->all_tiles, &all, sizeof(uint2), hipMemcpyHostToDevice);
    }
    e = e ? e : dev_alloc(&c->desc_dev, c->desc_bytes);
    e = e ? e : dev_alloc(&c->work_counter, static_cast<size_t>(kQueues) * kCounterStride);
    e = e ? e : dev_alloc(&c->assoc_hist, kAssocBuckets);
    e = e ? e : dev_alloc(&c->pairs, 1);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&c->desc_host), c->desc_bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&c->desc_done, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    for (hipEvent_t *ev : {&c->ev_start, &c->ev_vote0, &c->ev_vote1, &c->ev_end})
        if (e == hipSuccess)
            e = hipEventCreate(ev);
    if (e != hipSuccess) {
        const bool oom = e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation;
        hough_status st = oom ? HOUGH_ENOMEM : device_error(e, "hough_ctx_create");
        if (oom)
            g_last_error = "workspace allocation failed";
        free_ctx(c);
        return st;
    }
    *out = c;
    return HOUGH_OK;
}

void hough_ctx_destroy(hough_ctx *ctx) {
    if (!ctx)
        return;
    (void)hipDeviceSynchronize();
    free_ctx(ctx);
}

hough_status hough_set_launch(hough_ctx *ctx, int32_t which, int32_t rows, int32_t threads, int32_t split) {
    if (!ctx || (which != 0 && which != 1))
        return HOUGH_EINVAL;
    VoteShape s{rows, threads, split};
    if (which == 1 && split != 1)
        return HOUGH_EINVAL;
    if (!vote_shape_supported(s, ctx->u16, ctx->g.n_kappa, ctx->g.forward != 0))
        return HOUGH_EINVAL;
    if (which == 1 && batch_tiles_per_event(ctx, s, ctx->fused_batch) * static_cast<int64_t>(ctx->max_events) >
                          ctx->max_items)
        return HOUGH_EINVAL;
    if (ctx->desc_in_flight)
        HIP_TRY(hipEventSynchronize(ctx->desc_done));
    if (which == 0)
        ctx->shape_single = s;
    else
        ctx->shape_batch = s;
    drop_graphs(ctx);               // cached graphs embed the old shape
    ctx->last_hit_off.clear();      // the work list depends on the tile shape
    return HOUGH_OK;
}

hough_status hough_set_timing(hough_ctx *ctx, int32_t enable) {
    if (!ctx)
        return HOUGH_EINVAL;
    if (enable < 0 || enable > 2)
        return HOUGH_EINVAL;
    ctx->timing = enable != 0;
    ctx->count_pairs = enable == 2;
    ctx->timed_once = false;
    return HOUGH_OK;
}

hough_status hough_get_timing(hough_ctx *ctx, float *vote_ms, float *total_ms) {
    if (!ctx || !ctx->timed_once)
        return HOUGH_EINVAL;
    HIP_TRY(hipEventSynchronize(ctx->ev_end));
    float v = 0.0f, t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&v, ctx->ev_vote0, ctx->ev_vote1));
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev_start, ctx->ev_end));
    if (vote_ms)
        *vote_ms = v;
    if (total_ms)
        *total_ms = t;
    return HOUGH_OK;
}

hough_status hough_get_work(hough_ctx *ctx, uint64_t *evaluated_pairs) {
    if (!ctx || !ctx->timed_once || !ctx->count_pairs || !evaluated_pairs)
        return HOUGH_EINVAL;
    HIP_TRY(hipEventSynchronize(ctx->ev_end));
    unsigned long long v = 0;
    HIP_TRY(hipMemcpy(&v, ctx->pairs, sizeof v, hipMemcpyDeviceToHost));
    *evaluated_pairs = v;
    return HOUGH_OK;
}

hough_status hough_get_launch(const hough_ctx *ctx, int32_t which, int32_t *rows, int32_t *threads,
                              int32_t *split) {
    if (!ctx || (which != 0 && which != 1))
        return HOUGH_EINVAL;
    const VoteShape &s = which == 0 ? ctx->shape_single : ctx->shape_batch;
    if (rows)
        *rows = s.rows;
    if (threads)
        *threads = s.threads;
    if (split)
        *split = s.split;
    return HOUGH_OK;
}

hough_status hough_vote(hough_ctx *ctx, const float *x, const float *y, int32_t n_hits, void *acc,
                        uint64_t *n_votes, void *stream) {
    if (!ctx || !acc || n_hits < 0 || n_hits > ctx->max_hits)
        return HOUGH_EINVAL;
    if (n_hits > 0 && (!x || !y))
        return HOUGH_EINVAL;
    if (ctx->u16 && n_hits > 65535)
        return HOUGH_EINVAL;
    if (reinterpret_cast<uintptr_t>(acc) & 3u)
        return HOUGH_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto *nv = reinterpret_cast<unsigned long long *>(n_votes);
    const VoteShape &vs = ctx->shape_single;
    if (nv)
        HIP_TRY(launch_prep(nullptr, 1, nv, s));
    HIP_TRY(hit_prep(ctx, vs, false, x, y, n_hits, nullptr, s));
    HIP_TRY(launch_vote_single(ctx->g, ctx->u16, vs, vote_inputs(ctx, vs, false), n_hits,
                               static_cast<uint32_t *>(acc), nv, s));
    return HOUGH_OK;
}

hough_status hough_vertices(hough_ctx *ctx, const hough_vertex_grid *vgrid, int32_t n_events,
                            const hough_cand *cands, const int64_t *cand_off, const int32_t *n_found,
                            int32_t sorted_lists, int32_t track_threshold, int32_t vertex_threshold,
                            hough_cand *vout, const int64_t *vout_off, int32_t *n_vertices, int32_t *vacc,
                            void *stream) {
    if (!ctx || !vgrid || n_events < 1 || !cand_off || !n_found || !vout_off || !n_vertices || !vout)
        return HOUGH_EINVAL;
    if (!cands)
        return HOUGH_EINVAL;
    const hough_vertex_grid &vg = *vgrid;
    if (vg.n_x < 1 || vg.n_y < 1 || !vg.x_centre || !vg.y_centre)
        return HOUGH_EINVAL;
    if (!vertex_grid_supported(vg.n_x, vg.n_y)) {
        set_last_error("hough_vertices: vertex grid beyond 16384 cells, 4096 survivors or the LDS of a workgroup");
        return HOUGH_EINVAL;
    }
    HIP_TRY(launch_vertices(ctx->g, vg, n_events, reinterpret_cast<const Cand *>(cands), cand_off, n_found,
                            track_threshold, vertex_threshold, sorted_lists, reinterpret_cast<Cand *>(vout), vout_off,
                            n_vertices, vacc, static_cast<hipStream_t>(stream)));
    return HOUGH_OK;
}

hough_status hough_associate(hough_ctx *ctx, const float *x, const float *y, int32_t n_hits,
                             const hough_cand *cands, const int32_t *n_cands, int32_t cands_cap, int32_t min_votes,
                             int32_t *pairs, int64_t cap, uint64_t *n_pairs, void *stream) {
    if (!ctx || n_hits < 0 || cands_cap < 0 || cap < 0 || !n_cands || !n_pairs)
        return HOUGH_EINVAL;
    if ((n_hits > 0 && (!x || !y)) || (cands_cap > 0 && !cands) || (cap > 0 && !pairs))
        return HOUGH_EINVAL;
    if (reinterpret_cast<uintptr_t>(n_pairs) & 7u)
        return HOUGH_EINVAL;
    if (n_hits > ctx->max_hits)
        return HOUGH_EINVAL;
    HIP_TRY(launch_associate(ctx->g, x, y, n_hits, reinterpret_cast<const Cand *>(cands), n_cands, cands_cap,
                             min_votes, ctx->cell_map, ctx->cell_bits, ctx->hits, ctx->assoc_hist, pairs, cap,
                             reinterpret_cast<unsigned long long *>(n_pairs), ctx->cull_ok,
                             static_cast<hipStream_t>(stream)));
    return HOUGH_OK;
}

hough_status hough_peaks(hough_ctx *ctx, const void *acc, int32_t threshold, hough_cand *out, int32_t cap,
                         int32_t *n_found, void *stream) {
    if (!ctx || !acc || !n_found || cap < 0 || (cap > 0 && !out))
        return HOUGH_EINVAL;
    if (reinterpret_cast<uintptr_t>(acc) & 3u)
        return HOUGH_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SortWork w = sort_work(ctx, false);
    w.out = out;
    w.cap = cap;
    w.n_found = n_found;
    HIP_TRY(launch_prep(ctx->state, 1, nullptr, s));
    HIP_TRY(launch_peaks(ctx->g, ctx->u16, static_cast<const uint32_t *>(acc), 1, threshold, w, s));
    HIP_TRY(launch_sort(w, 1, s));
    return HOUGH_OK;
}

hough_status hough_vote_batch(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off, const float *x,
                              const float *y, void *acc, uint64_t *n_votes, void *stream) {
    if (check_batch(ctx, n_events, hit_off, x, y) != HOUGH_OK || !acc)
        return HOUGH_EINVAL;
    if (reinterpret_cast<uintptr_t>(acc) & 3u)
        return HOUGH_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool changed = false;
    hough_status st = stage_descriptors(ctx, n_events, hit_off, nullptr, false, &changed);
    if (st != HOUGH_OK)
        return st;
    DevDesc dd = device_descriptors(ctx);
    if (changed) {
        HIP_TRY(hipMemcpyAsync(ctx->desc_dev, ctx->desc_host, ctx->desc_bytes, hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ctx->desc_done, s));
        ctx->desc_in_flight = true;
    }
    const VoteShape &vs = ctx->shape_batch;
    auto *nv = reinterpret_cast<unsigned long long *>(n_votes);
    HIP_TRY(launch_prep_batch(ctx->state, ctx->max_events, &dd.hdr->n_events, nv, ctx->work_counter, s));
    HIP_TRY(hit_prep(ctx, vs, false, x, y, hit_off[n_events], nullptr, s));
    HIP_TRY(launch_vote_batch(ctx->g, ctx->u16, false, vs, vote_inputs(ctx, vs, false), dd.desc, &dd.hdr->queues,
                              dd.items, ctx->max_items, ctx->work_counter, ctx->cus * vote_groups_per_cu(vs, ctx->g.n_kappa),
                              static_cast<uint32_t *>(acc), nv, nullptr, 0, s));
    return HOUGH_OK;
}

}  // extern "C"

namespace {

// hough_event_batch, with packed lists when cand_start is given.
hough_status event_batch(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off, const float *x, const float *y,
                         int32_t threshold, void *acc, hough_cand *cands, const int64_t *cand_off,
                         int64_t *cand_start, int32_t *n_found, uint64_t *n_votes, void *stream) {
    if (!cand_off || !n_found || check_batch(ctx, n_events, hit_off, x, y) != HOUGH_OK)
        return HOUGH_EINVAL;
    if (cand_start && (reinterpret_cast<uintptr_t>(cand_start) & 7u))
        return HOUGH_EINVAL;
    if (cand_off[0] != 0)
        return HOUGH_EINVAL;
    for (int32_t e = 0; e < n_events; ++e)
        if (cand_off[e + 1] < cand_off[e] || cand_off[e + 1] - cand_off[e] > 0x7fffffffLL)
            return HOUGH_EINVAL;
    if (cand_off[n_events] > 0 && !cands)
        return HOUGH_EINVAL;
    if (acc && (reinterpret_cast<uintptr_t>(acc) & 3u))
        return HOUGH_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);

    bool changed = false;
    hough_status st = stage_descriptors(ctx, n_events, hit_off, cand_off, ctx->fused_batch, &changed);
    if (st != HOUGH_OK)
        return st;

    const int64_t bucket = hit_bucket(hit_off[n_events]);
    const uint32_t key_mask = batch_key_mask(ctx, n_events, hit_off);
    GraphKey key{x, y, acc, cands, n_found, n_votes, cand_start, threshold, bucket, key_mask};
    // Executable graphs are kept per key, least recently used evicted first: a
    // served lane sees batches of many sizes (hit buckets, sort passes), and
    // a capture costs far more than the replay it saves.
    hipGraphExec_t exec = nullptr;
    for (size_t k = 0; k < ctx->graphs.size(); ++k)
        if (ctx->graphs[k].key == key) {
            const GraphEntry hit = ctx->graphs[k];
            ctx->graphs.erase(ctx->graphs.begin() + static_cast<std::ptrdiff_t>(k));
            ctx->graphs.push_back(hit);
            exec = hit.exec;
            break;
        }
    if (ctx->timing) {
        // Direct launches with events around the vote (no graph).
        if (changed)
            HIP_TRY(hipMemcpyAsync(ctx->desc_dev, ctx->desc_host, ctx->desc_bytes, hipMemcpyHostToDevice, s));
        HIP_TRY(enqueue_batch(ctx, s, x, y, threshold, acc, cands, n_found, n_votes, cand_start, bucket, key_mask,
                              true));
        ctx->timed_once = true;
        if (changed) {
            HIP_TRY(hipEventRecord(ctx->desc_done, s));
            ctx->desc_in_flight = true;
        }
        return HOUGH_OK;
    }
    if (!exec) {
        hipStream_t cs = ctx->capture_stream;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipMemcpyAsync(ctx->desc_dev, ctx->desc_host, ctx->desc_bytes, hipMemcpyHostToDevice, cs);
        if (ce == hipSuccess)
            ce = enqueue_batch(ctx, cs, x, y, threshold, acc, cands, n_found, n_votes, cand_start, bucket, key_mask,
                               false);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (ce != hipSuccess) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return device_error(ce, "hough_event_batch capture");
        }
        if (ee != hipSuccess)
            return device_error(ee, "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess)
            return device_error(ie, "hipGraphInstantiate");
        if (ctx->graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back(GraphEntry{key, exec});
    }
    HIP_TRY(hipGraphLaunch(exec, s));
    // Every replay's first node copies the pinned block, changed or not, so
    // the block may be rewritten only after the latest replay has read it.
    HIP_TRY(hipEventRecord(ctx->desc_done, s));
    ctx->desc_in_flight = true;
    return HOUGH_OK;
}

}  // namespace

extern "C" {

hough_status hough_event_batch(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off, const float *x,
                               const float *y, int32_t threshold, void *acc, hough_cand *cands,
                               const int64_t *cand_off, int32_t *n_found, uint64_t *n_votes, void *stream) {
    return event_batch(ctx, n_events, hit_off, x, y, threshold, acc, cands, cand_off, nullptr, n_found, n_votes,
                       stream);
}

hough_status hough_event_batch_packed(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off, const float *x,
                                      const float *y, int32_t threshold, void *acc, hough_cand *cands,
                                      const int64_t *cand_off, int64_t *cand_start, int32_t *n_found,
                                      uint64_t *n_votes, void *stream) {
    if (!cand_start)
        return HOUGH_EINVAL;
    return event_batch(ctx, n_events, hit_off, x, y, threshold, acc, cands, cand_off, cand_start, n_found, n_votes,
                       stream);
}

}  // extern "C"
