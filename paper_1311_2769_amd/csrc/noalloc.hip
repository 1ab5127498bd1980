// hough_event_noalloc: one event's vote, peak search and sort without a
// context and without allocating device memory.  The scratch the kernels need
// (hit records, tile words or ranges, the table flag, the per-event state and
// the sort buffers) lives in one file-scope device array of fixed size; the
// caller passes the inputs and the outputs.  The kernels are the ones of
// hough_vote and hough_peaks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "hough.h"
#include "hough_impl.h"

using namespace hough;

namespace {

constexpr size_t kScratchBytes = HOUGH_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The scratch array.  Host code never passes its name to a kernel or a copy:
// in host code the name is a host-side stand-in, not the device address.  The
// address on each device comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t scratch_on_device(int device, unsigned char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

size_t align256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

// Byte offsets of the scratch regions for one event of n_hits hits.
struct Layout {
    size_t flag, state, hits, ranges, stage, cnt0, hist, tmp0, total;
    int64_t bound;
    int32_t blocks0, hist_chunks;
};

Layout layout(const GridArgs &g, int64_t n_hits) {
    Layout L{};
    const int32_t pb = peak_blocks_per_event(g);
    L.bound = static_cast<int64_t>(pb) * peak_block_cap(g);
    L.blocks0 = pb;
    const int32_t cb = peak_blocks_per_chunk(g);
    const int64_t first = (pb + cb - 1) / cb;
    const int64_t later = (L.bound + kSortChunk - 1) / kSortChunk;
    L.hist_chunks = static_cast<int32_t>(std::max(first, later));
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at += align256(bytes > 0 ? bytes : 1);
        return here;
    };
    L.flag = take(sizeof(int32_t));
    L.state = take(sizeof(EventState));
    L.hits = take(static_cast<size_t>(n_hits) * sizeof(float4));
    L.ranges = take(static_cast<size_t>(g.n_d0) * static_cast<size_t>(ranges_entries(n_hits)) * sizeof(uint2));
    L.stage = take(static_cast<size_t>(L.bound) * sizeof(Cand));
    L.cnt0 = take(static_cast<size_t>(pb) * sizeof(int32_t));
    L.hist = take(static_cast<size_t>(L.hist_chunks) * kDigits * sizeof(uint32_t));
    L.tmp0 = take(static_cast<size_t>(L.bound) * sizeof(Cand));
    L.total = at;
    return L;
}

hough_status fail(hough_status st, const char *msg) {
    set_last_error(msg);
    return st;
}

hough_status hip_fail(hipError_t e, const char *what) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "hough_event_noalloc: %s: %s (%d)", what, hipGetErrorString(e),
                  static_cast<int>(e));
    set_last_error(buf);
    return HOUGH_EDEVICE;
}

}  // namespace

extern "C" hough_status hough_event_noalloc(const hough_grid *grid, const float *x, const float *y,
                                            int32_t n_hits, int32_t threshold, void *acc, hough_cand *out,
                                            int32_t cap, int32_t *n_found, uint64_t *n_votes, void *stream) {
    GridArgs g{};
    if (grid_setup(grid, &g) != HOUGH_OK)
        return fail(HOUGH_EINVAL, "hough_event_noalloc: invalid grid");
    if (!acc || !n_found || n_hits < 0 || cap < 0 || (cap > 0 && !out) || (n_hits > 0 && (!x || !y)))
        return fail(HOUGH_EINVAL, "hough_event_noalloc: null pointer or negative size");
    if ((reinterpret_cast<uintptr_t>(acc) & 3u) || (n_votes && (reinterpret_cast<uintptr_t>(n_votes) & 7u)))
        return fail(HOUGH_EINVAL, "hough_event_noalloc: misaligned accumulator or vote count");
    const bool u16 = grid->acc_type == HOUGH_ACC_U16;
    if (u16 && n_hits > 65535)
        return fail(HOUGH_EINVAL, "hough_event_noalloc: uint16 cells hold events of at most 65535 hits");
    // A 32-row d0-grid tile of at most 512 threads is compiled for three
    // workgroups per CU and keeps a few loop-invariant values in scratch,
    // which the runtime may have to grow on its first launch: this entry
    // point takes 1,024 threads there, whose kernel needs no scratch.
    const int32_t rows = default_tile_rows(g, u16);
    const VoteShape vs{rows, (g.d0 && rows <= 32) ? 1024 : 512, u16 ? 1 : 4};
    if (!vote_shape_supported(vs, u16, g.n_kappa, g.forward != 0))
        return fail(HOUGH_EINVAL, "hough_event_noalloc: kappa rows too long for an LDS tile");
    const Layout L = layout(g, n_hits);
    if (L.total > kScratchBytes)
        return fail(HOUGH_EINVAL, "hough_event_noalloc: event and grid need more than the "
                                  "HOUGH_NOALLOC_SCRATCH_BYTES of scratch");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (device < 0 || device >= kMaxDevices)
        return fail(HOUGH_EINVAL, "hough_event_noalloc: device ordinal beyond 63");
    unsigned char *base = nullptr;
    e = scratch_on_device(device, &base);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetSymbolAddress");

    auto *flag = reinterpret_cast<int32_t *>(base + L.flag);
    auto *state = reinterpret_cast<EventState *>(base + L.state);
    auto *hits = reinterpret_cast<float4 *>(base + L.hits);
    auto *ranges = reinterpret_cast<uint2 *>(base + L.ranges);
    const TileGeom tg = vote_tile_geom(g, vs, false);
    const bool masks = tg.tiles <= kMaskTiles;

    VoteInputs in{};
    in.hits = hits;
    in.ranges = ranges;
    in.range_stride = masks ? tile_word_stride(n_hits) : n_hits;
    in.range_step = 1;
    in.mask_mode = masks ? 1 : 0;

    SortWork w{};
    w.s0.stage = reinterpret_cast<Cand *>(base + L.stage);
    w.s0.cnt0 = reinterpret_cast<int32_t *>(base + L.cnt0);
    w.s0.n_blocks0 = L.blocks0;
    w.s0.cap0 = peak_block_cap(g);
    w.s0.cb = peak_blocks_per_chunk(g);
    w.hist = reinterpret_cast<uint32_t *>(base + L.hist);
    w.hist_chunks = L.hist_chunks;
    w.tmp0 = reinterpret_cast<Cand *>(base + L.tmp0);
    w.tmp1 = w.s0.stage;
    w.bound = L.bound;
    w.state = state;
    w.out = out;
    w.cap = cap;
    w.n_found = n_found;
    // A cell takes at most one vote per hit, so only the sort-key digits of
    // counts up to n_hits can differ.
    const int64_t most = u16 ? std::min<int64_t>(n_hits, 0xffff) : n_hits;
    uint32_t mask = 0;
    while (mask < 0x7fffffffu && static_cast<int64_t>(mask) < most)
        mask = (mask << 1) | 1u;
    w.key_mask = mask;

    hipStream_t s = static_cast<hipStream_t>(stream);
    auto *nv = reinterpret_cast<unsigned long long *>(n_votes);
    // Every region that must start at a known value is written by a kernel of
    // this call: the flag by the table check, the state and the vote count by
    // prep, the hit records and tile entries by hit_prep, the histograms by
    // the peak search (zeroed first when blocks share them).
    e = launch_table_check(g.cos_phi, g.sin_phi, g.n_phi, flag, s);
    if (e == hipSuccess)
        e = launch_prep(state, 1, nv, s);
    if (e == hipSuccess)
        e = launch_hit_prep(g, tg, x, y, n_hits, nullptr, hits, ranges, in.range_stride, true, masks, flag, s);
    if (e == hipSuccess)
        e = launch_vote_single(g, u16, vs, in, n_hits, static_cast<uint32_t *>(acc), nv, s);
    if (e == hipSuccess)
        e = launch_peaks(g, u16, static_cast<const uint32_t *>(acc), 1, threshold, w, s);
    if (e == hipSuccess)
        e = launch_sort(w, 1, s);
    if (e != hipSuccess)
        return hip_fail(e, "launch");
    return HOUGH_OK;
}
