// Internal declarations shared by the HIP sources of libhough (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "hough.h"

namespace hough {

// ---------------------------------------------------------------------------
// Sort geometry: candidates are ordered by an LSD radix sort over 8-bit digits
// of key = 0x7fffffff - votes (so ascending keys = descending votes); the
// stable passes keep the ascending-cell order in which the peak search emits
// them.  Only the digits in which the event's keys differ are sorted.
// ---------------------------------------------------------------------------
constexpr int kDigits = 256;
constexpr int kMaxPasses = 4;
constexpr int kSortChunk = 4096;      // elements per chunk in passes >= 1
constexpr int kSortThreads = 256;
constexpr int kScanThreads = 1024;

struct Cand {
    int32_t votes;
    int32_t cell;
};
static_assert(sizeof(Cand) == sizeof(hough_cand), "candidate layout");

__host__ __device__ inline uint32_t sort_key(int32_t votes) {
    return static_cast<uint32_t>(static_cast<int64_t>(0x7fffffff) - static_cast<int64_t>(votes));
}

// Per-event state of one call, reset by the prep kernel.
struct EventState {
    uint32_t key_min;
    uint32_t key_max;
    int32_t n_found;
    int32_t passes;       // LSD passes this event needs (>= 1), set by the pass-0 scan
};

// Per-event descriptor uploaded by hough_event_batch.
struct EventDesc {
    int64_t hit_begin;
    int64_t hit_end;
    int64_t cand_begin;   // output slice of the caller's candidate array
    int32_t cand_cap;
    int32_t pad_;
};

// A unit of batched vote work: one phi0 tile of one event.
struct WorkItem {
    int32_t event;
    int32_t tile;         // tile index inside the event (d0 slice major)
};

// Work queues of a persistent batched vote, one per XCD: workgroups are
// dispatched to the XCDs in turn (workgroup i on XCD i mod kQueues), so the
// workgroups of queue q share one L2, and all tiles of an event sit in one
// queue -- its hit records are fetched into one L2 rather than into every
// XCD's.  Queue q is items [begin[q], begin[q] + len[q]) of the work list (the
// queues back to back); a workgroup whose queue is empty takes work from the
// next queues in turn.
constexpr int kQueues = 8;
constexpr int kCounterStride = 32;    // int32s between queue counters: each on a 128-byte line of its own
struct QueueDesc {
    int32_t begin[kQueues];
    int32_t len[kQueues];
};

// Grid in the form the kernels take it.
struct GridArgs {
    const float *cos_phi;
    const float *sin_phi;
    const float *d0;      // nullptr for 2D
    int32_t n_d0, n_phi, n_kappa;
    float kappa_min, kappa_scale;
    int32_t row_dwords;   // dwords per (d0, phi0) row in global memory
    int32_t bin_bits;     // kappa_scale >= 1 and kappa_min != +0: the vote's unsigned range test is exact
    float near_band;      // 2E rounded up (vote_near_band): fast hits take the approximate bins; or -1: exact only
    float kf_off;         // RN(E - kappa_min kappa_scale), the approximate bins' offset
    float kscale2;        // 2 kappa_scale, the 3D approximate bins' slope
    int32_t straight;     // straight-line family: kappa := u (hit records (x, y, 1, 1)), the last axis is d0
    int32_t forward;      // forward-hemisphere option: a vote also needs x cos + y sin > 0
    int64_t cells;        // cells per event
    int64_t acc_dwords;   // dwords per event accumulator
};

// Where the first-pass candidate lists of every event live.  List (block) b
// of event e holds cnt0[e*n_blocks0 + b] candidates at
// stage + (e*n_blocks0 + b)*cap0; first-pass chunk c is blocks
// [c*cb, (c+1)*cb).
struct Stage0 {
    Cand *stage;
    int32_t *cnt0;
    int32_t n_blocks0;
    int32_t cap0;
    int32_t cb;
};

struct SortWork {
    Stage0 s0;
    uint32_t *hist;           // [events][hist_chunks][256], offsets in place after a scan
    int32_t hist_chunks;
    Cand *tmp0;               // [events][bound]
    Cand *tmp1;               // [events][bound] (aliases stage, which is dead after pass 0)
    int64_t bound;            // max candidates per event
    EventState *state;
    const EventDesc *desc;    // per-event output slices, or nullptr
    hough_cand *out;          // caller's candidate array
    int32_t cap;              // used when desc == nullptr (one event)
    int32_t *n_found;         // caller's [events]
    uint32_t key_mask;        // sort-key bits that can differ within an event (sets the passes)
    const int32_t *n_events_dev;  // batch: live event count on the device, or nullptr
    int64_t *cand_start;      // batch, packed lists: [events+1] list offsets written after the
                              // first scan (each list follows the previous one), or nullptr
};

// Hit inputs of a vote launch, as written by hit_prep: one record per hit
// and, with culling, two tile ranges per hit and d0 slice.
struct VoteInputs {
    const float4 *hits;        // [n] (x, y, z, w): see launch_hit_prep
    const uint2 *ranges;       // [n_d0][range_stride] tile ranges per hit, or one all-tiles entry
    int64_t range_stride;      // 0 with the all-tiles entry
    int32_t range_step;        // 1 with ranges, 0 with the all-tiles entry
    int32_t mask_mode;         // ranges holds transposed tile words (culling on, at most kMaskTiles tiles)
};

// A tile range packs first | count << 16 (tile indices of one d0 slice,
// cyclic; 15-bit count); count 0 is empty and kAllTiles covers every tile.
// Bit 31 of a hit's second range is kFastDiv: every phi0 row of that (hit,
// d0 slice) has its 3D quotient operands in the range of vote_math.h.
constexpr uint32_t kAllTiles = 0x7fffu << 16;
// With at most kMaskTiles tiles T per slice the buffer holds instead, per d0
// slice and 64-hit chunk of the record array, T + 1 transposed 64-bit words:
// word t has bit k set when hit 64 chunk + k can vote in tile t, word T when
// that (hit, slice) has the kFastDiv property.  Word (l, t, chunk) sits at
// (l tile_word_stride + chunk) (T + 1) + t -- the words of one chunk side by
// side, so hit_prep stores them at once -- 8 bytes like a range pair, so a
// buffer of ranges_entries(max_hits) entries per slice holds either form.
constexpr int32_t kMaskTiles = 63;
constexpr uint32_t kFastDiv = 1u << 31;
inline int64_t tile_word_stride(int64_t max_hits) { return (max_hits + 63) / 64; }
inline int64_t ranges_entries(int64_t max_hits) { return max_hits + 64; }

// Tile geometry of a vote launch: tile t of a slice owns phi0 rows
// [t*stride, min((t+1)*stride, n_phi)); with halo it also votes the row
// before and the row after (cyclically), for the fused peak search.
struct TileGeom {
    int32_t tiles;
    int32_t stride;
    int32_t halo;
};

// Launch shape of a vote kernel.
struct VoteShape {
    int32_t rows;     // phi0 rows per tile
    int32_t threads;  // workgroup size
    int32_t split;    // hit chunks per tile (single-event vote only)
};

// ---------------------------------------------------------------------------
// Launchers (return hipSuccess or the first launch error).
// ---------------------------------------------------------------------------
bool vote_shape_supported(const VoteShape &s, bool u16, int32_t n_kappa, bool forward);
size_t vote_lds_bytes(const VoteShape &s, int32_t n_kappa);
// Constants of the approximate bins (vote_math.h): E is twice the derived
// bound of |kf1 - (kf + E)| on |kf| <= n_kappa + 2; *band = 2E rounded up and
// *off = RN(E - kappa_min kappa_scale).  False (and the exact quotient only)
// when the grid is outside the range the bound covers.
bool vote_near_band(const GridArgs &g, float *band, float *off);
int32_t vote_tiles_per_slice(const GridArgs &g, const VoteShape &s, bool fused);
// Workgroups of launch shape s that fit one CU at once (LDS and wavefronts):
// the persistent batch launches that many per CU.
int32_t vote_groups_per_cu(const VoteShape &s, int32_t n_kappa);
// Slice units of a vote launch: uint16 grids with a d0 axis take their d0
// slices in pairs (one LDS tile counts the cells of both), others one at a
// time.  A launch has units x tiles_per_slice tiles per event.
inline int32_t vote_slice_units(const GridArgs &g, bool u16) {
    return (u16 && g.d0) ? (g.n_d0 + 1) / 2 : g.n_d0;
}
TileGeom vote_tile_geom(const GridArgs &g, const VoteShape &s, bool fused);
int32_t fused_chunk_cap(const GridArgs &g, const VoteShape &s);

// The rules of hough_ctx_create for a grid, and its kernel form (EINVAL when
// the grid is rejected).  api.hip.
hough_status grid_setup(const hough_grid *grid, GridArgs *out);
// Default tile height of a grid's vote kernels.
int32_t default_tile_rows(const GridArgs &g, bool u16);

hipError_t launch_prep(EventState *state, int32_t n_events, unsigned long long *n_votes,
                       hipStream_t stream);
// Batch form: state of all max_events slots, n_votes of the live events, work counter.
// work_counter: kQueues counters kCounterStride int32s apart, all zeroed.
hipError_t launch_prep_batch(EventState *state, int32_t max_events, const int32_t *n_events_dev,
                             unsigned long long *n_votes, int32_t *work_counter, hipStream_t stream);
hipError_t launch_zero(uint32_t *p, int64_t n_dwords, hipStream_t stream);
// Per-hit preparation of a vote launch with tile geometry tg.  hits[h] =
// (x, y, r2/2, w) for 2D hits whose quotient may use the hoisted division
// (div_fast and r2/2 in range), where w is the refined 1/(r2/2), times
// kappa_scale when the grid takes approximate bins (near_band > 0); else
// (x, y, r2, 0).  Straight-line hits are (x, y, 1, 1), or (x, y, 1,
// kappa_scale) with approximate bins.  With
// ranges: ranges[l*range_stride + h] holds the two tile ranges of slice l
// outside which hit h cannot vote.  n_hits_dev, when given, overrides n_hits
// (which then only sizes the grid).  table_ok, when given, is a device flag
// read by the kernel: zero makes every entry take every tile and every record
// the division operator, as if div_fast were false (a phi0 table that does not
// hold the bin centres); nullptr means the caller has checked the table.
hipError_t launch_hit_prep(const GridArgs &g, const TileGeom &tg, const float *x, const float *y, int64_t n_hits,
                           const int64_t *n_hits_dev, float4 *hits, uint2 *ranges, int64_t range_stride,
                           bool div_fast, bool masks, const int32_t *table_ok, hipStream_t stream);
// Device check of a phi0 table against the bin centres (j + 1/2) 2 pi / n_phi
// (angle within 1e-6 rad, norm within 1e-6 of 1, n_phi <= 32768): writes 1 or
// 0 to *ok.  One workgroup; allocates nothing.
hipError_t launch_table_check(const float *cos_phi, const float *sin_phi, int32_t n_phi, int32_t *ok,
                              hipStream_t stream);

// One event: hits [0, n_hits).
// pairs (measurement only): when given, the launch adds the (hit, phi0 row)
// pairs it evaluates -- staged hits times tile rows -- to *pairs.
hipError_t launch_vote_single(const GridArgs &g, bool u16, const VoteShape &s, const VoteInputs &in,
                              int32_t n_hits, uint32_t *acc, unsigned long long *n_votes, hipStream_t stream,
                              unsigned long long *pairs = nullptr);
// Many events: tile work items over events described by desc; the queues
// (live item counts) are read on the device.  With work counters (reset
// beforehand) the launch is persistent: persistent_groups workgroups pull
// items from their XCD's queue, then from the others; without, workgroup i
// takes item i of the queues back to back.
// fused (2D int32 only): tiles also search their interior rows for peaks into
// the staging lists of *w; acc may then be nullptr.
hipError_t launch_vote_batch(const GridArgs &g, bool u16, bool fused, const VoteShape &s, const VoteInputs &in,
                             const EventDesc *desc, const QueueDesc *queues, const WorkItem *items,
                             int32_t max_items, int32_t *work_counter, int32_t persistent_groups, uint32_t *acc,
                             unsigned long long *n_votes, const SortWork *w, int32_t threshold,
                             hipStream_t stream, unsigned long long *pairs = nullptr);

int32_t peak_blocks_per_event(const GridArgs &g);
int32_t peak_block_cap(const GridArgs &g);
int32_t peak_blocks_per_chunk(const GridArgs &g);
hipError_t launch_peaks(const GridArgs &g, bool u16, const uint32_t *acc, int32_t n_events,
                        int32_t threshold, const SortWork &w, hipStream_t stream);
hipError_t launch_sort(const SortWork &w, int32_t n_events, hipStream_t stream);

// Second transform (vertex.hip).  Grids need n_x * n_y <= kVtxMaxCells and a
// survivor bound ceil(n_x/2) * ceil(n_y/2) <= kVtxMaxPeaks (LDS-resident).
constexpr int32_t kVtxMaxCells = 16384;
constexpr int32_t kVtxMaxPeaks = 4096;
int32_t vertex_sort_size(int32_t n_x, int32_t n_y);
bool vertex_grid_supported(int32_t n_x, int32_t n_y);   // the limits above and the workgroup's LDS
hipError_t launch_vertices(const GridArgs &g, const hough_vertex_grid &vg, int32_t n_events, const Cand *cands,
                           const int64_t *cand_off, const int32_t *n_found, int32_t track_threshold,
                           int32_t vertex_threshold, int32_t sorted, Cand *vout, const int64_t *vout_off,
                           int32_t *n_vertices, int32_t *vacc, hipStream_t stream);

// ---------------------------------------------------------------------------
// Launch-shape cache (tune.hip).
// ---------------------------------------------------------------------------
struct TuneEntry {
    std::string device;   // architecture / compute units, e.g. "gfx950/256"
    int n_d0 = 0, n_phi = 0, n_kappa = 0;
    int acc = 0;          // hough_acc_type
    int which = 0;        // 0 single event, 1 batch
    int hits_log2 = 0;    // hit count rounded up to a power of two
    int rows = 0, threads = 0, split = 1;
    double ms = 0.0;
};
int tune_hits_log2(int64_t hits);
bool tune_parse(const char *line, TuneEntry *e);
std::string tune_format(const TuneEntry &e);
// Entry of key (device, grid, acc, which) nearest to key.hits_log2; false if none.
bool tune_lookup(const char *path, const TuneEntry &key, TuneEntry *out);
bool tune_append(const char *path, const TuneEntry &e);
std::string device_tag(int device);
// The explicit path, else $HOUGH_TUNE_CACHE, else nullptr.
const char *tune_cache_path(const char *opt);

}  // namespace hough

// The grid a context was created for (api.hip).
void ctx_grid(const hough_ctx *ctx, hough_grid *out);
// Set this thread's hough_last_error() text (api.hip).
void set_last_error(const char *msg);

