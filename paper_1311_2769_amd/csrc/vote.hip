// Hough vote kernels for gfx950.
//
// Section 3: every hypothesis starts with zero votes and every hit adds one
// vote to each hypothesis it lies on; Section 4: the work for each hit is
// independent of the others.
//
// Layout.  The accumulator of one d0 slice is cut into tiles of 32, 64 or 128
// consecutive phi0 rows.  A workgroup owns one tile as a private LDS
// accumulator.  A lane keeps the cos/sin of its phi0 rows and the slice's d0
// in registers.  2D: 16 lanes span the rows of a 32- or 64-row tile (32 of a
// 128-row one), each lane taking every hit for 2-4 rows, so a wavefront
// evaluates four hits (two) per instruction and each staged record read
// serves several rows.  3D: a lane owns one row, 64 rows of one hit or 32
// rows of two hits per instruction.  The LDS tile is kappa-major (dword
// (kappa, row) at kappa*rows + row): the lanes of one hit are distinct rows,
// so its LDS atomics fall in distinct banks whatever kappa bins it produces.  Every lane adds on every evaluation: a lane whose
// hit casts no vote in its row adds into one spare kappa column past the
// grid, which keeps the loop free of branches.  The finished tile is flushed
// to HBM, lanes again across rows -- no global atomics on the accumulator --
// and the vote count is reduced per wavefront and added once per workgroup.
//
// Hits.  hit_prep_kernel writes one record per hit (x, y and the hit's
// denominator terms) and, per d0 slice, the two cyclic ranges of tiles
// outside which the hit cannot vote.  The wavefronts of a tile take the
// event's records in chunks of 64, round robin, each on its own: a lane loads
// one record of the wavefront's next chunk while the current one is
// evaluated, and only the hits whose ranges hold the tile are staged, in the
// wavefront's own LDS region.  Lane groups read staged hits one iteration
// ahead of their votes; the fewer than 4G hits left over after whole
// iterations are carried into the wavefront's next chunk, so only its last
// chunk has a partial iteration.  The workgroup meets at a barrier only when
// the tile is zeroed and when its votes are in.
//
// Culling.  A hit can only vote in the phi0 rows where its curvature lies in
// the kappa range: two arcs of phi0 per d0 slice.  hit_prep_kernel computes
// both arcs, widened by bounds on every fp32 rounding of the vote arithmetic
// (see below), and converts them to the tiles whose voted rows meet them.
// Which votes are cast is still decided only by the exact fp32 test, so
// culling changes no result.
//
// Arithmetic is the fp32 definition in hough.h, op for op; this file is
// compiled with -ffp-contract=off.  r2 = x*x + y*y is computed with the same
// operations in hit_prep_kernel.  For the 2D grid (d0 == +0) the numerator
// 2*(u - 0) equals 2*u and the denominator (r2 - 0*u) + 0*0 equals r2 for every
// finite u, and both forms give NaN or an out-of-range kf otherwise, so the 2D
// kernels divide 2*u by r2.  Hits whose r2/2 lies in the range of vote_math.h
// carry (x, y, r2/2, refined 1/(r2/2)), are staged at the front of the block
// and are evaluated as u / (r2/2) with the hoisted division: the same real
// quotient as 2u / r2, so the same correctly rounded result.  The others
// carry (x, y, r2, 0), are staged at the back and divide with the operator.
// 3D hits carry (x, y, r2, 0); those whose (hit, d0 slice) hit_prep_kernel
// marks kFastDiv are staged at the front and divide with the operator's own
// sequence minus its operand scaling and special-value fix-up, which are
// no-ops when every operand is in the range of vote_math.h (rcp, two
// refinement FMAs, then quot_apply): 8 instead of 11 operations.
//
// uint16 accumulators of a 2D grid count in int32 LDS cells like int32 ones
// and are packed two cells per dword (even kappa bin in the low half) when
// the tile is flushed; on a d0 grid one LDS dword counts the same cell of two
// slices (slice pairs, below) and the flush repacks them the same way.
// Counts fit because a cell receives at most one vote per hit and u16 events
// hold at most 65535 hits.
//
// Fused peak search (2D int32 batches).  Tiles then overlap by two rows: a
// tile votes S interior rows plus one halo row on each side, finds the local
// maxima of its interior rows straight from LDS and appends them in cell
// order to its staging list; the accumulator need not reach HBM at all.
#pragma clang fp contract(off)

#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

#include "hough_impl.h"
#include "peak_tile.h"
#include "vote_math.h"
#include "arc_math.h"

namespace hough {
namespace {

struct VoteArgs {
    GridArgs g;
    const float4 *hits;         // hit records (x, y, z, w)
    const uint2 *ranges;        // [n_d0][range_stride] tile ranges per hit; or one all-tiles entry (step 0)
    int64_t range_stride;
    int32_t range_step;         // 1 with ranges, 0 without
    int32_t mask_mode;          // ranges holds the transposed tile words (see hit_prep_kernel)
    int32_t n_hits;             // single event
    int32_t split;              // single event: hit chunks per tile
    int32_t tiles_per_slice;
    int32_t tile_stride;        // tile t starts at row t*tile_stride + tile_off
    int32_t tile_off;           // 0, or -1 for fused tiles
    const EventDesc *desc;      // batch: per-event hit ranges
    const WorkItem *items;      // batch: tile list, or nullptr for a single event
    const QueueDesc *queues;    // batch: the list's work queues (device)
    int32_t *work_counter;      // batch, persistent: next item of each queue (kCounterStride apart)
    uint32_t *acc;              // dwords; fused batches may pass nullptr
    unsigned long long *n_votes;
    SortWork w;                 // fused: staging lists
    int32_t threshold;          // fused
    unsigned long long *pairs;  // measurement: (hit, row) pairs evaluated, added per tile, or nullptr
};

// Each wavefront stages the hit records of its own chunks (chunk c of a
// tile's hit range belongs to wavefront c mod NW, one record per lane) in a
// region of its own: fast hits from the front, after a carried remainder of
// fewer than kCarryMax, slow ones downwards from kRegionSlow, and kCarryMax
// slots of slack after that for the reads a lane group issues past the end of
// a list (values that are never used).
constexpr int kChunk = 64;
constexpr int kCarryMax = 16;                      // 4 x (hits per wavefront instruction, at most 4)
constexpr int kRegionSlow = kChunk + kCarryMax;
constexpr int kRegion = kRegionSlow + kCarryMax;

template <int NT>
struct TileScratch {
    float4 hits[NT / 64][kRegion];   // each wavefront's staged hits
    CompactScratch<NT> sc;
    int32_t cnt[NT];                 // fused peak search: candidates per (row, kappa segment)
    int32_t wave_tot[NT / 64];
    unsigned long long red[NT / 64];
    int32_t next_item;
    unsigned long long pairs;        // measurement: pairs this workgroup evaluated, added once at its end
};

__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Vote hits [h_begin, h_end) of event e into tile t of slice unit l, then
// either flush it (unfused) or search its interior rows for peaks (fused).
// A slice unit is one d0 slice, or with uint16 cells on a d0 grid two
// (slice pairs: slices 2l and 2l + 1, the second absent past the grid).
//
// Slice pairs.  A uint16 event holds at most 65535 hits and a cell takes at
// most one vote per hit, so an LDS dword can count the cell (kappa, row) of
// both slices: the first in its low half, the second in its high half (adds
// of 1 and of 0x10000 never carry into each other).  The tile then covers
// two slices in the LDS of one, every staged hit serves both, and u =
// y c - x s of a (hit, row) is computed once for the two bins.
template <bool U16, bool D3, int ROWS, int NT, bool FUSED, bool FWD>
__device__ void vote_tile(const VoteArgs &a, int e, int l, int t, int64_t h_begin, int64_t h_end,
                          uint32_t *__restrict__ acc_event, bool atomic_flush, unsigned long long *n_votes,
                          uint32_t *lds, TileScratch<NT> &ts) {
    // Lanes across rows.  2D: 16 (32 for 128-row tiles), so that a lane
    // takes every staged hit for 2-4 rows and one record read serves them
    // all; 3D: one row per lane (slice pairs measured slower with several).
    constexpr int RL = D3 ? (ROWS < 64 ? ROWS : 64) : (ROWS / 4 < 16 ? 16 : ROWS / 4);
    constexpr int HPW = 64 / RL;                // hits per wavefront instruction
    constexpr int RPT = ROWS / RL;              // rows per lane
    constexpr int NW = NT / 64;
    constexpr int G = HPW;                      // lane groups of a wavefront
    constexpr int stride = ROWS;                // dwords per LDS kappa column
    static_assert(4 * G <= kCarryMax, "staging slack");
    const GridArgs &g = a.g;
    const int tid = threadIdx.x;
    const int n_phi = g.n_phi;
    const int T = a.tiles_per_slice;
    const int first = t * a.tile_stride + a.tile_off;      // may be -1 for a fused tile
    int len, s_here = 0;
    if constexpr (FUSED) {
        s_here = min(a.tile_stride, n_phi - t * a.tile_stride);
        len = s_here + 2;
    } else {
        len = min(ROWS, n_phi - first);
    }

    // n_kappa columns plus one spare column that takes the no-vote adds
    const int nk_cols = g.n_kappa;
    for (int i = tid; i < (nk_cols + 1) * stride; i += NT)
        lds[i] = 0u;
    if constexpr (FUSED) {
        for (int i = tid; i < kDigits; i += NT)
            ts.sc.hist[i] = 0u;
    }

    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rlane = lane % RL;
    const int hsub = lane / RL;
    float c[RPT], s[RPT];
    int rowoff[RPT];
    const float nkf = static_cast<float>(g.n_kappa);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = rlane + RL * i;
        const bool live = r < len;
        int j = first + r;
        if (j < 0)
            j += n_phi;
        if (j >= n_phi)
            j -= n_phi;
        if (!live)
            j = 0;
        // rows past the tile get NaN constants: their kf is NaN, which no bin accepts
        c[i] = live ? g.cos_phi[j] : __builtin_nanf("");
        s[i] = live ? g.sin_phi[j] : __builtin_nanf("");
        rowoff[i] = r;
    }
    constexpr bool SP = U16 && D3;               // slice pairs
    const int l0 = SP ? 2 * l : l;               // the (first) d0 slice
    const bool has1 = SP && l0 + 1 < g.n_d0;     // the pair's second slice exists
    const float d = D3 ? g.d0[l0] : 0.0f;
    // an absent second slice takes d = NaN: every bin of it misses
    const float d_1 = has1 ? g.d0[l0 + 1] : __builtin_nanf("");
    // Let the row constants land now: the memory counter is in order, so a
    // first use inside the hit loop would also wait for the hit prefetches.
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
    const float d2 = 2.0f * d;
    const float dd = d * d;
    const float d2_1 = 2.0f * d_1;
    const float dd_1 = d_1 * d_1;
    const float kmin = g.kappa_min;
    const float kscale = g.kappa_scale;
    const int trash = nk_cols;                                 // bin index of the spare column
    // ... held in a VGPR so that the select below is a single v_cndmask
    int trash_v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(trash_v) : "s"(trash));
    const float4 *__restrict__ hrec = a.hits;
    const uint2 *__restrict__ rrow = a.ranges + static_cast<int64_t>(l0) * a.range_stride;
    const uint2 *__restrict__ rrow1 = has1 ? rrow + a.range_stride : rrow;
    const int64_t rmask = a.range_step ? -1 : 0;   // per-hit ranges, or the one all-tiles entry
    const bool mask_mode = a.mask_mode != 0;

    // Kappa bin of one staged hit (x, y, z, w) at row i of this lane: the bin
    // to add to, which is the spare column when the hit casts no vote there.
    // fast (2D only): z = r2/2 and w its refined reciprocal.  Otherwise z = r2
    // and the operator divides.
    //
    // The range test 0 <= kf < n_kappa.  With bits (GridArgs::bin_bits) it is
    // one unsigned minimum: non-negative floats order like their bit patterns,
    // and negative numbers and NaNs have larger patterns, so
    // v = min(bits(kf), bits(n_kappa + 1/2)) is kf itself on [+0, n_kappa +
    // 1/2) and n_kappa + 1/2 elsewhere; truncated, it is kf's bin when kf votes
    // and n_kappa -- the spare column -- when it does not.  This needs kf never to be -0,
    // which the oracle would accept: kf = (kappa - kappa_min) * kappa_scale is
    // -0 only for kappa = -0 with kappa_min = +0 (the context stores -0
    // instead, which changes no vote) or when a nonzero difference (at least
    // 2^-149) times kappa_scale rounds to zero, impossible for kappa_scale >= 1.
    // (The approximate bins clamp the same way, kf_clamp.)
    const uint32_t lim_bits = __float_as_uint(nkf + 0.5f);
    auto bin_of = [&](float kf, int i, bool valid, auto bits) -> int {
        if constexpr (decltype(bits)::value) {
            const uint32_t b = valid ? __float_as_uint(kf) : 0xffffffffu;
            return static_cast<int>(__uint_as_float(min(b, lim_bits)));
        } else {
            const bool ok = valid && kf >= 0.0f && kf < nkf;
            return ok ? static_cast<int>(kf) : trash_v;
        }
    };
    // Forward option: the row counts only when the hit lies ahead,
    // x c + y s > 0 in binary32 (NaN rows past the tile fail it too).
    auto ahead = [&](const float4 &h, int i, bool valid, auto fwd) -> bool {
        if constexpr (decltype(fwd)::value) {
            const float w = h.x * c[i] + h.y * s[i];
            return valid && w > 0.0f;
        } else {
            return valid;
        }
    };
    // Slice constants (d, 2d, d*d) of the unit's first or second slice.
    auto sconst = [&](auto sl) {
        if constexpr (decltype(sl)::value)
            return make_float3(d_1, d2_1, dd_1);
        else
            return make_float3(d, d2, dd);
    };
    using S0 = std::false_type;
    using S1 = std::true_type;
    auto bin = [&](const float4 &h, int i, bool valid, auto fast, auto bits, auto fwd, auto sl) -> int {
        valid = ahead(h, i, valid, fwd);
        const float u = h.y * c[i] - h.x * s[i];
        float kappa;
        if constexpr (D3) {
            const float3 sc = sconst(sl);
            const float d = sc.x, d2 = sc.y, dd = sc.z;
            const float den = (h.z - d2 * u) + dd;
            if constexpr (decltype(fast)::value) {
                // In range, 2(u - d) / den = 2 ((u - d) / den) exactly (scaling a
                // normal number by 2 is exact, so the correctly rounded
                // quotients agree), and kappa - kappa_min = fma(2, q, -kappa_min)
                // with its one rounding (2q is exact).  The quotient runs the
                // operator's own steps with operand scaling elided.
                const float q = quot_apply(u - d, den, quot_recip(den));
                const float kf = __builtin_fmaf(2.0f, q, -kmin) * kscale;
                return bin_of(kf, i, valid, bits);
            } else {
                kappa = (2.0f * (u - d)) / den;
            }
        } else if constexpr (decltype(fast)::value) {
            kappa = quot_apply(u, h.z, h.w);
        } else {
            kappa = (2.0f * u) / h.z;
        }
        const float kf = (kappa - kmin) * kscale;
        return bin_of(kf, i, valid, bits);
    };
    // Approximate bins with exact redos (fast hits, GridArgs::near_band > 0;
    // the bound is in vote_math.h): kf1 from one FMA, and the lanes whose kf1
    // falls in the band above an integer take the exact kf.  num: the
    // quotient's numerator (u in 2D), kept for the redo.
    const float near_band = g.near_band;
    float kf_off = g.kf_off;
    const float kscale2 = g.kscale2;
    if constexpr (D3) {
        // the 3D FMA already takes kscale2 from a scalar register: keep the
        // offset in a vector one, or the compiler moves it there per hit pair
        asm volatile("v_mov_b32 %0, %1" : "=v"(kf_off) : "s"(g.kf_off));
    }
    auto bin_approx = [&](const float4 &h, int i, bool valid, auto bits, auto fwd, float &num, float &den,
                          bool &near, auto sl) -> int {
        valid = ahead(h, i, valid, fwd);
        const float u = h.y * c[i] - h.x * s[i];
        float kf1;
        if constexpr (D3) {
            const float3 sc = sconst(sl);
            const float d = sc.x, d2 = sc.y, dd = sc.z;
            num = u - d;
            den = (h.z - d2 * u) + dd;
            kf1 = kf_offset_3d(num, den, kscale2, kf_off);
        } else {
            num = u;
            kf1 = kf_offset_2d(u, h.w, kf_off);
        }
        const float v = kf_clamp(valid ? kf1 : __builtin_nanf(""), lim_bits);
        near = kf_in_band(v, near_band);
        return static_cast<int>(v);
    };
    auto bin_exact = [&](float num, float den, int i, bool valid, auto bits) -> int {
        return bin_of(D3 ? kf_exact_3d(num, den, kmin, kscale) : kf_exact_2d(num, den, kmin, kscale), i, valid, bits);
    };
    // 3D redo: num and den formed again from the record with bin_approx's
    // operations (the same fp32 values), so that they need not stay live
    // across the approximate bins of both hits and slices
    auto bin_exact_3d = [&](const float4 &h, int i, bool valid, auto bits, auto sl) -> int {
        const float u = h.y * c[i] - h.x * s[i];
        const float3 sc = sconst(sl);
        return bin_exact(u - sc.x, (h.z - sc.y * u) + sc.z, i, valid, bits);
    };
    auto vote = [&](int kk, int i, uint32_t one) { lds_add(&lds[kk * stride + rowoff[i]], one); };
    // Evaluate and vote two hits of this lane group (valid: the hit exists):
    // fast 0 the division operator, 1 the hoisted exact quotient, 2 the
    // approximate bins with exact redos.  With slice pairs each (hit, row)
    // takes a bin in both slices; u is computed once for the two (the same
    // operations on the same operands), and one wave-uniform branch redoes
    // the lanes of either slice.
    auto eval2 = [&](const float4 &ha, const float4 &hb, bool va, bool vb, auto fast, auto bits, auto fwd) {
        int ka[RPT], kb[RPT], ka1[RPT], kb1[RPT];
        if constexpr (decltype(fast)::value == 2) {
            float na[RPT], da[RPT], nb[RPT], db[RPT], na1[RPT], da1[RPT], nb1[RPT], db1[RPT];
            bool fa[RPT], fb[RPT], fa1[RPT], fb1[RPT];
            bool any = false;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                ka[i] = bin_approx(ha, i, va, bits, fwd, na[i], da[i], fa[i], S0{});
                kb[i] = bin_approx(hb, i, vb, bits, fwd, nb[i], db[i], fb[i], S0{});
                any |= fa[i] || fb[i];
                if constexpr (SP) {
                    ka1[i] = bin_approx(ha, i, va, bits, fwd, na1[i], da1[i], fa1[i], S1{});
                    kb1[i] = bin_approx(hb, i, vb, bits, fwd, nb1[i], db1[i], fb1[i], S1{});
                    any |= fa1[i] || fb1[i];
                }
            }
            // one wave-uniform branch for both hits, so their chains interleave
            if (__ballot(any)) {
                if constexpr (!D3) {
                    // the 2D denominator r2/2 is the hit's own
#pragma unroll
                    for (int i = 0; i < RPT; ++i) {
                        da[i] = ha.z;
                        db[i] = hb.z;
                    }
                }
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    if constexpr (D3) {
                        if (fa[i])
                            ka[i] = bin_exact_3d(ha, i, va, bits, S0{});
                        if (fb[i])
                            kb[i] = bin_exact_3d(hb, i, vb, bits, S0{});
                        if constexpr (SP) {
                            if (fa1[i])
                                ka1[i] = bin_exact_3d(ha, i, va, bits, S1{});
                            if (fb1[i])
                                kb1[i] = bin_exact_3d(hb, i, vb, bits, S1{});
                        }
                    } else {
                        if (fa[i])
                            ka[i] = bin_exact(na[i], da[i], i, va, bits);
                        if (fb[i])
                            kb[i] = bin_exact(nb[i], db[i], i, vb, bits);
                    }
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                ka[i] = bin(ha, i, va, fast, bits, fwd, S0{});
                kb[i] = bin(hb, i, vb, fast, bits, fwd, S0{});
                if constexpr (SP) {
                    ka1[i] = bin(ha, i, va, fast, bits, fwd, S1{});
                    kb1[i] = bin(hb, i, vb, fast, bits, fwd, S1{});
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            vote(ka[i], i, 1u);
            vote(kb[i], i, 1u);
            if constexpr (SP) {
                vote(ka1[i], i, 0x10000u);
                vote(kb1[i], i, 0x10000u);
            }
        }
    };
    // Staged hits [lo, hi) of this wavefront's region (lo, hi wave-uniform).
    // An iteration covers 2G consecutive hits: lane group hsub takes hits
    // it + hsub and it + G + hsub.  Two iterations per trip, the next pair
    // read before the current votes are cast (two register sets, no copies),
    // so waiting for a read never waits for atomics still in flight.  Whole
    // trips need no per-lane checks; a tail of fewer than 4G hits checks.
    float4 *region = ts.hits[wave];
    auto sweep_with = [&](int lo, int hi, auto fast, auto bits, auto fwd) {
        if (lo >= hi)
            return;
        const float4 *hp = region + hsub;
        int it = lo;
        float4 a0 = hp[it], b0 = hp[it + G];
        for (; it + 4 * G <= hi; it += 4 * G) {
            const float4 a1 = hp[it + 2 * G], b1 = hp[it + 3 * G];
            eval2(a0, b0, true, true, fast, bits, fwd);
            a0 = hp[it + 4 * G];
            b0 = hp[it + 5 * G];
            eval2(a1, b1, true, true, fast, bits, fwd);
        }
        if (it < hi) {
            const float4 a1 = hp[it + 2 * G], b1 = hp[it + 3 * G];
            eval2(a0, b0, it + hsub < hi, it + G + hsub < hi, fast, bits, fwd);
            if (it + 2 * G < hi)
                eval2(a1, b1, it + 2 * G + hsub < hi, it + 3 * G + hsub < hi, fast, bits, fwd);
        }
    };
    // (the forward option is a kernel of its own: its variants inlined here
    // beside the default ones cost the default kernel about 3 %)
    const bool bin_bits = g.bin_bits != 0;
    auto sweep = [&](int lo, int hi, auto fast) {
        if (bin_bits)
            sweep_with(lo, hi, fast, std::true_type{}, std::integral_constant<bool, FWD>{});
        else
            sweep_with(lo, hi, fast, std::false_type{}, std::integral_constant<bool, FWD>{});
    };
    // Is this tile in the cyclic tile range r?
    auto in_range = [&](uint32_t r) {
        int dt = t - static_cast<int>(r & 0xffffu);
        dt += dt < 0 ? T : 0;
        return dt < static_cast<int>((r >> 16) & 0x7fffu);
    };

    // Chunks: 64 hits at a multiple of 64 of the record array (the first and
    // last chunks of the range may hold other events' hits, which the range
    // mask drops); chunk g0 + wave + k NW belongs to this wavefront.  Its
    // lanes load the records of its next chunk (and the tile's word of it,
    // or the per-hit ranges) while the current one is evaluated; the kept
    // hits are staged in the wavefront's region and evaluated.  LDS
    // operations of one wavefront complete in order, so no barrier is needed
    // until the tile is done; fast hits short of a whole trip are carried
    // into the next chunk, so only the last chunk has a partial trip.
    // Record indices fit 32 bits (contexts hold at most 2^30 hits).
    const int hb = static_cast<int>(h_begin);
    const int he = static_cast<int>(h_end);
    const int g_stop = (he + 63) >> 6;
    const uint64_t *__restrict__ words = reinterpret_cast<const uint64_t *>(a.ranges);
    const int64_t ws = a.range_stride;
    int kept_here = 0;                           // hits this wavefront staged (pair counting only)
    lds_barrier();                               // the tile is zeroed
    auto chunks = [&](auto by_words) __attribute__((always_inline)) {
        constexpr bool W = decltype(by_words)::value;
        // With words, the word of a chunk is the same for every lane: loaded
        // as a vector value (through zero_v, a zero the compiler cannot see
        // through) and made scalar only where used, since a scalar copy right
        // after the load would wait for it -- and the records -- at once.
        int zero_v;
        asm volatile("v_mov_b32 %0, 0" : "=v"(zero_v));
        const int wstep = T + 1;                 // words of one chunk
        const int64_t w0 = static_cast<int64_t>(l0) * ws * wstep;
        const int64_t w1 = has1 ? w0 + ws * wstep : w0;   // a slice pair's second slice
        const uint2 *__restrict__ wtile = reinterpret_cast<const uint2 *>(words + w0 + t) + zero_v;
        const uint2 *__restrict__ wflag = reinterpret_cast<const uint2 *>(words + w0 + T) + zero_v;
        const uint2 *__restrict__ wtile1 = reinterpret_cast<const uint2 *>(words + w1 + t) + zero_v;
        const uint2 *__restrict__ wflag1 = reinterpret_cast<const uint2 *>(words + w1 + T) + zero_v;
        float4 ph = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        uint2 pr = make_uint2(0u, 0u);           // the tile's word of the chunk, or the hit's ranges
        uint2 pf = make_uint2(0u, 0u);           // 3D with words: the chunk's kFastDiv word
        uint2 pr1 = make_uint2(0u, 0u), pf1 = make_uint2(0u, 0u);   // the same of a pair's second slice
        // (always inlined, through a local: otherwise the 2D kernels kept the
        // prefetched records in a stack slot and waited for each load at once)
        auto fetch = [&](int gg) __attribute__((always_inline)) {
            const int h = min(max((gg << 6) + lane, hb), he - 1);
            ph = hrec[h];
            if constexpr (W) {
                pr = wtile[gg * wstep];
                if constexpr (D3)
                    pf = wflag[gg * wstep];
                if constexpr (SP) {
                    pr1 = wtile1[gg * wstep];
                    pf1 = wflag1[gg * wstep];
                }
            } else {
                pr = rrow[h & rmask];
                if constexpr (SP)
                    pr1 = rrow1[h & rmask];
            }
        };
        auto uniform64 = [](uint2 v) {
            const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v.x)));
            const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v.y)));
            return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
        };
        int gc = (hb >> 6) + wave;
        if (gc < g_stop)
            fetch(gc);
        int carry = 0;                           // fast hits carried into this chunk
        for (; gc < g_stop; gc += NW) {
            // lanes of the chunk inside [h_begin, h_end)
            const int lo = hb - (gc << 6);
            const int hi = he - (gc << 6);
            uint64_t inside = hi >= 64 ? ~0ull : (1ull << hi) - 1ull;
            if (lo > 0)
                inside &= ~((1ull << lo) - 1ull);
            // kept: the hit can vote in this tile (of either slice of a pair);
            // fast: its quotients take the fast form (in both slices)
            uint64_t K, F;
            if constexpr (W) {
                K = uniform64(pr);
                F = D3 ? uniform64(pf) : __ballot(ph.w != 0.0f);
                if constexpr (SP) {
                    K |= uniform64(pr1);
                    F &= uniform64(pf1);
                }
                K &= inside;
            } else {
                bool in = in_range(pr.x) || in_range(pr.y);
                bool fst = D3 ? (pr.y & kFastDiv) != 0u : ph.w != 0.0f;
                if constexpr (SP) {
                    in = in || in_range(pr1.x) || in_range(pr1.y);
                    fst = fst && (pr1.y & kFastDiv) != 0u;
                }
                K = __ballot(in) & inside;
                F = __ballot(fst);
            }
            const uint64_t mf = K & F;
            const uint64_t ms = K & ~F;
            kept_here += __popcll(K);
            const bool keep = ((K >> lane) & 1ull) != 0ull;
            const bool fast = ((F >> lane) & 1ull) != 0ull;
            const int slot = fast ? carry + rank_below(mf) : kRegionSlow - 1 - rank_below(ms);
            if (keep)
                region[slot] = ph;
            const int n_fast = carry + __popcll(mf);
            const int n_slow = __popcll(ms);
            const bool last = gc + NW >= g_stop;
            const int whole = last ? n_fast : n_fast - n_fast % (4 * G);
            if (!last)
                fetch(gc + NW);
            if (near_band > 0.0f)
                sweep(0, whole, std::integral_constant<int, 2>{});
            else
                sweep(0, whole, std::true_type{});
            sweep(kRegionSlow - n_slow, kRegionSlow, std::false_type{});
            carry = n_fast - whole;
            // the carried hits to the front (whole is 0 or at least 4G > carry:
            // the two ranges do not overlap)
            if (whole > 0 && lane < carry) {
                const float4 v = region[whole + lane];
                region[lane] = v;
            }
        }
    };
    if (hb < he) {
        if (mask_mode)
            chunks(std::true_type{});
        else
            chunks(std::false_type{});
    }
    lds_barrier();
    // Every staged hit is evaluated once per row of the tile (halo rows
    // included); rows past the grid take NaN constants and are not counted.
    // Summed in LDS; the workgroup adds its total to a.pairs when it ends.
    if (a.pairs && lane == 0 && kept_here > 0)
        __hip_atomic_fetch_add(&ts.pairs, static_cast<unsigned long long>(kept_here) *
                                              static_cast<unsigned long long>(has1 ? 2 * len : len),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);

    const int rd = g.row_dwords;
    unsigned long long votes = 0;
    // Post-vote work runs with lanes across rows (conflict-free LDS reads):
    // thread tid handles row rr = tid % ROWS over kappa segment tid / ROWS.
    constexpr int SEGS = NT / ROWS;
    static_assert(SEGS * ROWS == NT, "tile rows divide the workgroup");
    const int rr = tid % ROWS;
    const int seg = tid / ROWS;
    if constexpr (FUSED) {
        // Interior rows 1..s_here of the tile are phi0 rows j_first.. of slice 0.
        const int j_first = t * a.tile_stride;
        const int nk = g.n_kappa;
        const int32_t *col = reinterpret_cast<const int32_t *>(lds) + rr;   // column k of this row at col[k*stride]
        const int32_t thr = a.threshold;
        const int kseg = (nk + SEGS - 1) / SEGS;
        const int k_lo = min(nk, seg * kseg);
        const int k_hi = min(nk, k_lo + kseg);
        const bool row_ok = rr >= 1 && rr <= s_here;
        uint32_t *dst = (acc_event && row_ok) ? acc_event + static_cast<int64_t>(j_first + rr - 1) * rd : nullptr;

        // Scan cells (rr, k_lo..k_hi) in order with a sliding 3x3 window of
        // (row above, row, row below) columns k-1, k, k+1; kappa columns
        // outside the grid read as INT_MIN, so they never stop a peak.
        // Offsets (phi0, kappa) that are lexicographically negative -- the row
        // above, or this row at k-1 -- must be exceeded, the others reached.
        auto scan = [&](auto on_cell) {
            int32_t uA = INT_MIN, mA = INT_MIN, dA = INT_MIN;
            if (k_lo > 0) {
                const int32_t *q = col + (k_lo - 1) * stride;
                uA = q[-1];
                mA = q[0];
                dA = q[1];
            }
            const int32_t *q = col + k_lo * stride;
            int32_t uB = q[-1], mB = q[0], dB = q[1];
            auto cell = [&](int k, int32_t uC, int32_t mC, int32_t dC) {
                const int32_t above = max(max(uA, uB), max(uC, mA));
                const int32_t below = max(max(dA, dB), max(dC, mC));
                on_cell(k, mB, mB >= thr && mB > above && mB >= below);
                uA = uB;
                mA = mB;
                dA = dB;
                uB = uC;
                mB = mC;
                dB = dC;
            };
            const int k_stop = min(k_hi, nk - 1);
            int k = k_lo;
            for (; k < k_stop; ++k) {
                q += stride;
                cell(k, q[-1], q[0], q[1]);
            }
            if (k < k_hi)
                cell(k, INT_MIN, INT_MIN, INT_MIN);
        };

        // pass 1: peaks per (row, segment) as a bit mask, vote count and the
        // accumulator row if wanted
        uint64_t pm = 0;
        int mine = 0;
        if (row_ok && k_lo < k_hi) {
            scan([&](int k, int32_t v, bool pk) {
                votes += static_cast<uint32_t>(v);
                if (dst)
                    dst[k] = static_cast<uint32_t>(v);
                if (pk) {
                    ++mine;
                    if (k - k_lo < 64)
                        pm |= 1ull << (k - k_lo);
                }
            });
        }
        // exclusive offsets in cell order: (row, segment) pairs row-major
        const int order = rr * SEGS + seg;
        ts.cnt[order] = mine;
        lds_barrier();
        const int v_in = ts.cnt[tid];
        int incl = v_in;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off, 64);
            if (lane >= off)
                incl += o;
        }
        if (lane == 63)
            ts.wave_tot[wave] = incl;
        lds_barrier();
        int wpre = 0, total = 0;
#pragma unroll
        for (int wv = 0; wv < NW; ++wv) {
            const int c0 = ts.wave_tot[wv];
            wpre += wv < wave ? c0 : 0;
            total += c0;
        }
        lds_barrier();
        ts.cnt[tid] = wpre + incl - v_in;
        lds_barrier();
        // pass 2: write in cell order, histogram the first sort digit
        Cand *out = a.w.s0.stage + (static_cast<int64_t>(e) * a.w.s0.n_blocks0 + t) * a.w.s0.cap0;
        uint32_t kmin_key = 0xffffffffu, kmax_key = 0u;
        if (mine > 0) {
            int pos = ts.cnt[order];
            auto emit = [&](int k, int32_t v) {
                out[pos++] = Cand{v, (j_first + rr - 1) * nk + k};
                const uint32_t key = sort_key(v);
                atomicAdd(&ts.sc.hist[key & 0xffu], 1u);
                kmin_key = min(kmin_key, key);
                kmax_key = max(kmax_key, key);
            };
            if (k_hi - k_lo <= 64) {
                for (uint64_t m = pm; m; m &= m - 1) {
                    const int k = k_lo + __builtin_ctzll(m);
                    emit(k, col[k * stride]);
                }
            } else {
                scan([&](int k, int32_t v, bool pk) {
                    if (pk)
                        emit(k, v);
                });
            }
        }
        kmin_key = wave_min_u32(kmin_key);
        kmax_key = wave_max_u32(kmax_key);
        if (lane == 0) {
            ts.sc.red_min[wave] = kmin_key;
            ts.sc.red_max[wave] = kmax_key;
        }
        lds_barrier();
        uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
        for (int wv = 0; wv < NW; ++wv) {
            mn = min(mn, ts.sc.red_min[wv]);
            mx = max(mx, ts.sc.red_max[wv]);
        }
        publish_block<NT>(a.w, e, t, total, ts.sc, mn, mx);
    } else {
        const int kseg = (rd + SEGS - 1) / SEGS;
        const int w_lo = min(rd, seg * kseg);
        const int w_hi = min(rd, w_lo + kseg);
        if (SP && rr < len) {
            // slice pairs: each LDS dword holds the cell of both slices; the
            // uint16 rows of the two slices pair kappa bins 2wd and 2wd + 1
            uint32_t *dst0 = acc_event + (static_cast<int64_t>(l0) * n_phi + first + rr) * rd;
            uint32_t *dst1 = dst0 + static_cast<int64_t>(n_phi) * rd;
            for (int wd = w_lo; wd < w_hi; ++wd) {
                const uint32_t lo = lds[(2 * wd) * stride + rr];
                const uint32_t hi = lds[(2 * wd + 1) * stride + rr];
                votes += (lo & 0xffffu) + (lo >> 16) + (hi & 0xffffu) + (hi >> 16);
                const uint32_t v0 = (lo & 0xffffu) | (hi << 16);
                const uint32_t v1 = (lo >> 16) | (hi & 0xffff0000u);
                if (!atomic_flush) {
                    dst0[wd] = v0;
                    if (has1)
                        dst1[wd] = v1;
                } else {
                    if (v0)
                        atomicAdd(&dst0[wd], v0);
                    if (has1 && v1)
                        atomicAdd(&dst1[wd], v1);
                }
            }
        } else if (rr < len) {
            uint32_t *dst = acc_event + (static_cast<int64_t>(l) * n_phi + first + rr) * rd;
            for (int wd = w_lo; wd < w_hi; ++wd) {
                uint32_t v;
                if constexpr (U16) {
                    const uint32_t lo = lds[(2 * wd) * stride + rr];
                    const uint32_t hi = lds[(2 * wd + 1) * stride + rr];
                    votes += lo + hi;
                    v = lo | (hi << 16);
                } else {
                    v = lds[wd * stride + rr];
                    votes += v;
                }
                if (!atomic_flush)
                    dst[wd] = v;
                else if (v)
                    atomicAdd(&dst[wd], v);
            }
        }
    }
    if (n_votes) {
        const unsigned long long wsum = wave_sum_u64(votes);
        if (lane == 0)
            ts.red[wave] = wsum;
        lds_barrier();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int wv = 0; wv < NW; ++wv)
                tot += ts.red[wv];
            if (tot)
                atomicAdd(n_votes, tot);
        }
    }
    lds_barrier();   // the LDS tile and scratch are reused by the next item
}

// Waves per SIMD the compiler must leave room for.  The 32-row d0-grid tiles
// take about 48 KiB of LDS, so three workgroups of 512 threads (six waves
// per SIMD) fit a CU when the kernel keeps to 80 VGPRs; left alone it took
// 114 and two fitted (the displaced batch's vote 2.15 -> 2.02 ms with
// three).  A 2D workgroup of 1,024 threads holds its CU's LDS alone; kept to
// 96 VGPRs (five waves per SIMD, 127 left alone, no spills) it leaves room
// for the waves of the kernels that run between two votes -- the next
// batch's hit_prep, the sort passes -- which then start while its last
// items finish (batched 2D step 1.289 -> 1.270 ms).  Other shapes keep the
// default.
template <bool D3, int ROWS, int NT>
constexpr int vote_min_waves() {
    return (D3 && ROWS <= 32 && NT <= 512) ? 6 : (!D3 && NT == 1024) ? 5 : 1;
}

template <bool U16, bool D3, int ROWS, int NT, bool FUSED, bool FWD>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(vote_min_waves<D3, ROWS, NT>(), 8)))
void vote_kernel(VoteArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ TileScratch<NT> ts;
    const int T = a.tiles_per_slice;
    // measurement: the workgroup's evaluated pairs, one global add at its end
    if (a.pairs && threadIdx.x == 0)
        ts.pairs = 0ull;
    auto add_pairs = [&]() {
        if (a.pairs) {
            lds_barrier();
            if (threadIdx.x == 0 && ts.pairs)
                atomicAdd(a.pairs, ts.pairs);
        }
    };

    if (a.items == nullptr) {
        const int tile = blockIdx.x;
        const int l = tile / T;
        const int t = tile - l * T;
        const int64_t n = a.n_hits;
        const int64_t per = (n + a.split - 1) / a.split;
        const int64_t hb = static_cast<int64_t>(blockIdx.y) * per;
        const int64_t he = min(n, hb + per);
        vote_tile<U16, D3, ROWS, NT, FUSED, FWD>(a, 0, l, t, hb, he, a.acc, a.split > 1, a.n_votes, lds, ts);
        add_pairs();
        return;
    }
    const QueueDesc *qd = a.queues;
    int32_t it = blockIdx.x;
    int q = blockIdx.x % kQueues;     // this XCD's queue (thread 0 keeps track)
    int tried = 0;
    for (;;) {
        if (a.work_counter) {
            if (threadIdx.x == 0) {
                int32_t item = -1;
                while (tried < kQueues) {
                    const int32_t k = atomicAdd(&a.work_counter[q * kCounterStride], 1);
                    if (k < qd->len[q]) {
                        item = qd->begin[q] + k;
                        break;
                    }
                    q = q + 1 < kQueues ? q + 1 : 0;      // empty: the next queue
                    ++tried;
                }
                ts.next_item = item;
            }
            lds_barrier();
            it = ts.next_item;
            lds_barrier();
        } else if (it >= qd->begin[kQueues - 1] + qd->len[kQueues - 1]) {
            it = -1;
        }
        if (it < 0) {
            add_pairs();
            return;
        }
        const WorkItem wi = a.items[it];
        const EventDesc ev = a.desc[wi.event];
        const int l = wi.tile / T;
        const int t = wi.tile - l * T;
        uint32_t *acc_e = a.acc ? a.acc + static_cast<int64_t>(wi.event) * a.g.acc_dwords : nullptr;
        vote_tile<U16, D3, ROWS, NT, FUSED, FWD>(a, wi.event, l, t, ev.hit_begin, ev.hit_end, acc_e, false,
                                            a.n_votes ? a.n_votes + wi.event : nullptr, lds, ts);
        if (!a.work_counter) {
            add_pairs();
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-hit preparation: the hit record, and the two phi0 arcs per d0 slice
// where a hit may vote, as ranges of tiles.
//
// Bound used (angles in radians, K' = max |kappa edge| (1 + 1e-3)).  If a vote
// is cast, the fp32 curvature kappa_c lies within max |kappa edge| (1 + 2^-19).
// kappa_c rounds num_c / den_c, where num_c = 2(u_c - d) to 2^-24 relative,
// u_c = y c - x s to r 2^-20 absolute (fp32 products, and fp32 cos/sin of the
// bin centre), and den_c equals r^2 - 2 d u_c + d^2 to 2^-21 (r + |d|)^2
// absolute.  The exact denominator |h - P0|^2 is at least (r - |d|)^2, so when
// |r - |d|| >= 0.03 (r + |d|) its relative error is at most 2^-21 / 0.03^2 <
// 5.3e-4, kappa(u_c) = 2(u_c - d)/(r^2 + d^2 - 2 d u_c) is within relative
// 5.4e-4 of kappa_c, and |kappa(u_c)| <= K'.  On |u| <= r the function
// kappa(u) is continuous and monotone (its derivative has the sign of
// r^2 - d^2; its pole (r^2 + d^2) / (2 d) lies at least 0.0018 r beyond
// |u| = r under the same condition), and its inverse
// u(k) = (k (r^2 + d^2) + 2 d) / (2 (1 + k d)) is continuous and monotone on
// [-K', K'] when K' |d| < 1, so u_c lies between u(-K') and u(K') and
// sin(phi_h - phi0) lies between s(-K') and s(K'), s(k) = u(k) / r, widened
// by 1e-5.
//
// hit_prep_kernel evaluates s(-+K) in fp32 as (2d -+ K rr) (1/(2r)) / (1 -+ K d)
// with K = K' rounded up to fp32 (a larger K only widens the interval),
// rr = r2 + d^2, r = sqrt(r2) and the reciprocals from arc_rcp.  One rounding
// per operation (2^-24 relative, 2^-23 for arc_rcp, 3 2^-24 for r) bounds the
// error of either end by (K rr + 2|d|) (1/r) w^2 17 2^-25, w = 1 / (1 - K|d|);
// the interval is widened by 1e-5 + 2^-18 (K rr + 2|d|) (1/r) w^2, more than
// four times that on top of the 1e-5.  The fp32 tests r in [2^-30, 2^30],
// |d| <= 2^30, |r - |d|| >= 0.0301 (r + |d|) and K |d| <= 0.99 imply the real
// conditions above; a hit or slice that fails them, or whose ends are not
// finite, gets the full circle.
//
// The arcs of phi0 whose sine lies in the widened interval (from
// phi_h = hit_angle(x, y) and arc_asin of its clamped ends) are widened by
// kArcTol = 1e-4 rad, which covers the library angle error (at most
// kArcAngleErrMax each, checked by hough_selftest_angles), the fp32 angle
// sums (|angle| <= 2.5 pi) and the fp32 scaling to rows, and then by one row
// on each side.  The phi0 table must hold the bin centres
// (j + 1/2) 2 pi / n_phi (checked when the context is created; otherwise no
// ranges are used).
//
// An arc of rows (start, length; length 0: empty, n_phi: the full circle) is
// turned into the cyclic range of tiles that vote any of its rows: the tile
// owning its first row (or, with halos, the tile before when that row is the
// first of its tile) through the tile owning its last row (or the tile after
// when that row is the last of its tile).  n_phi is limited to 32768, so the
// tile count fits the 16-bit fields.
// ---------------------------------------------------------------------------

struct PrepArgs {
    const float *x;
    const float *y;
    int64_t n_hits;
    const int64_t *n_hits_dev;  // batch: live hit count (overrides n_hits), or nullptr
    float4 *hits;
    uint2 *ranges;              // nullptr: no culling
    int64_t range_stride;
    const float *d0;            // nullptr for 2D
    int32_t n_phi;
    int32_t n_d0;
    int32_t tiles, tile_stride, halo;
    uint32_t stride_magic;      // ceil(2^32 / tile_stride), 0 when tile_stride == 1
    int32_t div_fast;
    float w_scale;              // kappa_scale with approximate bins, else 1 (hit record w)
    float kabs;                 // K' rounded up to fp32 (may be +inf)
    int32_t straight;           // straight-line family: records (x, y, 1, 1), arcs from the d0 range
    int32_t forward;            // forward-hemisphere option: the first arc only
    float dlo, dhi;             // straight: the d0 range, rounded outwards
    int32_t mask_mode;          // write transposed tile words instead of ranges (tiles <= kMaskTiles)
    const int32_t *table_ok;    // device flag: the phi0 table holds the bin centres (else no arcs and no
                                // fast division), or nullptr when the host has checked the table
};

// Transpose of the 64 x 64 bit matrix whose row L is lane L's m: lane t
// gets bit L set exactly when bit t of lane L's m is set.  Butterfly steps
// j = 32, 16, .., 1 swap the off-diagonal j x j blocks of every 2j x 2j
// block: a lane with bit j clear keeps its columns with bit j clear and takes
// its partner's (lane ^ j) as the columns above; a lane with bit j set keeps
// the columns with bit j set and takes its partner's from below.
template <int J>
__device__ __forceinline__ void transpose_step(uint32_t &lo, uint32_t &hi, int lane) {
    // ds_swizzle in bit mode: lane ^ J within each 32-lane half
    constexpr int kPattern = 0x1f | (J << 10);
    // the columns with bit J clear, within each 32-bit word
    constexpr uint32_t kKeep = J == 16 ? 0x0000ffffu : J == 8 ? 0x00ff00ffu : J == 4 ? 0x0f0f0f0fu
                               : J == 2 ? 0x33333333u : 0x55555555u;
    const uint32_t ylo = static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(static_cast<int>(lo), kPattern));
    const uint32_t yhi = static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(static_cast<int>(hi), kPattern));
    const bool up = (lane & J) != 0;
    const uint32_t keep = up ? ~kKeep : kKeep;
    const uint32_t slo = up ? ylo >> J : ylo << J;
    const uint32_t shi = up ? yhi >> J : yhi << J;
    lo = (lo & keep) | (slo & ~keep);
    hi = (hi & keep) | (shi & ~keep);
}

__device__ __forceinline__ uint64_t lane_transpose(uint64_t m, int lane) {
    uint32_t lo = static_cast<uint32_t>(m), hi = static_cast<uint32_t>(m >> 32);
    const uint32_t plo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(lo), 32));
    const uint32_t phi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(hi), 32));
    if (lane & 32)
        lo = phi;
    else
        hi = plo;
    transpose_step<16>(lo, hi, lane);
    transpose_step<8>(lo, hi, lane);
    transpose_step<4>(lo, hi, lane);
    transpose_step<2>(lo, hi, lane);
    transpose_step<1>(lo, hi, lane);
    return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
}

// The tiles of a cyclic range as bits of a mask (T <= kMaskTiles).
__device__ __forceinline__ uint64_t range_bits(uint32_t r, int T) {
    const int cnt = static_cast<int>((r >> 16) & 0x7fffu);
    const int first = static_cast<int>(r & 0xffffu);
    if (cnt == 0)
        return 0ull;
    if (cnt >= T)
        return (1ull << T) - 1ull;
    if (first + cnt <= T)
        return ((1ull << cnt) - 1ull) << first;
    return (((1ull << (T - first)) - 1ull) << first) | ((1ull << (first + cnt - T)) - 1ull);
}

// Rows whose centres (j + 1/2) 2 pi / n lie in [phi_a, phi_b], widened by
// kArcTol and one row on each side; sc = n / (2 pi) in fp32.
__device__ __forceinline__ uint32_t pack_arc(float phi_a, float phi_b, int n, float sc) {
    const float lo = ceilf((phi_a - kArcTol) * sc - 0.5f) - 1.0f;
    const float hi = floorf((phi_b + kArcTol) * sc - 0.5f) + 1.0f;
    if (hi < lo)
        return 0u;
    const float rows = hi - lo + 1.0f;
    if (rows >= static_cast<float>(n))
        return static_cast<uint32_t>(n) << 16;
    int start = static_cast<int>(lo);          // |lo| <= 1.25 n + 2
    while (start < 0)
        start += n;
    while (start >= n)
        start -= n;
    return static_cast<uint32_t>(start) | (static_cast<uint32_t>(rows) << 16);
}

__device__ __forceinline__ uint32_t tile_range(uint32_t arc, const PrepArgs &p) {
    const int n = p.n_phi;
    const int len = static_cast<int>(arc >> 16);
    if (len == 0)
        return 0u;
    if (len >= n)
        return kAllTiles;
    const int S = p.tile_stride;
    const int T = p.tiles;
    const int start = static_cast<int>(arc & 0xffffu);
    const int end_u = start + len - 1;                 // unwrapped, < 2n
    const int end = end_u >= n ? end_u - n : end_u;
    int lo = p.stride_magic ? div_small(start, p.stride_magic) : start;
    if (p.halo && start == lo * S)
        lo -= 1;                                       // the tile before votes it as its upper halo
    const int oe = p.stride_magic ? div_small(end, p.stride_magic) : end;
    int hi = (end_u >= n ? T : 0) + oe;
    if (p.halo && end == oe * S + min(S, n - oe * S) - 1)
        hi += 1;                                       // the tile after votes it as its lower halo
    const int cnt = hi - lo + 1;
    if (cnt >= T)
        return kAllTiles;
    if (lo < 0)
        lo += T;
    return static_cast<uint32_t>(lo) | (static_cast<uint32_t>(cnt) << 16);
}

constexpr int kPrepSlices = 8;   // d0 slices per hit_prep thread (per-hit terms computed once)

__global__ __launch_bounds__(256) void hit_prep_kernel(PrepArgs p) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = p.n_hits_dev ? *p.n_hits_dev : p.n_hits;
    // With tile words every lane of a wavefront takes part in the ballots,
    // live or not; dead lanes read nothing and set no bit.
    const bool live = i < n;
    if (!p.mask_mode && !live)
        return;
    if (p.mask_mode && __ballot(live) == 0ull)
        return;                              // no word of this wavefront's chunk exists
    const float xf = live ? p.x[i] : 0.0f;
    const float yf = live ? p.y[i] : 0.0f;
    const float r2 = xf * xf + yf * yf;
    const int l_begin = blockIdx.y * kPrepSlices;
    // Arcs and the fast division rest on a table of bin centres; without one
    // every (hit, slice) takes every tile and the division operator.
    const bool table = p.table_ok == nullptr || *p.table_ok != 0;
    if (l_begin == 0 && live) {
        float4 rec = make_float4(xf, yf, r2, 0.0f);
        if (p.straight) {
            // the 2D fast path then computes kappa = quot_apply(u, 1, 1) = u
            // exactly (q0 = u, both remainders 0; a -0 may come out +0, which
            // lands in the same bin), and the approximate bins fma(u, w, off)
            // with w = kappa_scale
            rec = make_float4(xf, yf, 1.0f, p.w_scale);
        } else if (p.div_fast && table && p.d0 == nullptr) {
            const float half = 0.5f * r2;
            if (quot_den_ok(half))
                rec = make_float4(xf, yf, half, quot_recip(half) * p.w_scale);
        }
        p.hits[i] = rec;
    }
    if (!p.ranges)
        return;
    // The (hit, slice) entry: per-hit ranges, or (mask_mode) the hit's bit in
    // the transposed words of its 64-hit chunk g = i / 64 -- word t of slice l
    // has bit k set when hit 64 g + k can vote in tile t, word T (the tile
    // count) when its 3D quotients take the fast division.  Lane t < T writes
    // tile t's word, lane T the flags.
    const int lane = threadIdx.x & 63;
    auto emit = [&](int l, uint2 out) {
        if (!p.mask_mode) {
            p.ranges[static_cast<int64_t>(l) * p.range_stride + i] = out;
            return;
        }
        const int T = p.tiles;
        const uint64_t m = live ? (range_bits(out.x, T) | range_bits(out.y & ~kFastDiv, T)) : 0ull;
        // lane t < T takes tile t's word (the transposed masks), lane T the flags
        const uint64_t flags = __ballot(live && (out.y & kFastDiv) != 0u);
        const uint64_t tw = lane_transpose(m, lane);
        const uint64_t mine = lane == T ? flags : tw;
        uint64_t *words = reinterpret_cast<uint64_t *>(p.ranges);
        if (lane <= T)
            words[(static_cast<int64_t>(l) * p.range_stride + (i >> 6)) * (T + 1) + lane] = mine;
    };
    if (!table) {
        const int l_stop = p.straight ? 1 : min(l_begin + kPrepSlices, p.d0 ? p.n_d0 : 1);
        for (int l = l_begin; l < l_stop; ++l)
            emit(l, make_uint2(kAllTiles, 0u));
        return;
    }
    const float r = sqrtf(r2);
    const bool r_ok = r >= 0x1.0p-30f && r <= 0x1.0p30f;     // false for NaN
    const float inv_r = arc_rcp(r_ok ? r : 1.0f);
    const float half_inv_r = 0.5f * inv_r;
    const float ph = hit_angle(xf, yf);
    const float K = p.kabs;
    const float sc = static_cast<float>(p.n_phi) * 0.159154943f;
    const float pi = 3.14159274f;
    const int l_end = min(l_begin + kPrepSlices, p.d0 ? p.n_d0 : 1);
    // the sine interval -> two arcs -> two tile ranges.  The first arc,
    // phi_h - phi0 in [asin(lo), asin(hi)] within [-pi/2, pi/2], holds the
    // rows where the hit lies ahead (cos(phi_h - phi0) >= 0); the second its
    // mirror.  The forward option keeps the first alone: the vote's own
    // ahead test decides the rows within the arc widening of +-pi/2, where
    // fp32 may call a row either way (within 1e-6 rad of the real boundary).
    const bool fwd = p.forward != 0;
    auto arcs = [&](float slo, float shi) {
        if (!(isfinite(slo) && isfinite(shi)))
            return make_uint2(kAllTiles, 0u);   // full circle
        if (slo > 1.0f || shi < -1.0f)
            return make_uint2(0u, 0u);
        if (!fwd && slo <= -1.0f && shi >= 1.0f)
            return make_uint2(kAllTiles, 0u);
        const float alo = arc_asin(fmaxf(slo, -1.0f));
        const float ahi = arc_asin(fminf(shi, 1.0f));
        const float pm = ph - pi;
        return make_uint2(tile_range(pack_arc(ph - ahi, ph - alo, p.n_phi, sc), p),
                          fwd ? 0u : tile_range(pack_arc(pm + alo, pm + ahi, p.n_phi, sc), p));
    };
    if (p.straight) {
        // Straight lines: a vote needs u_c in [dlo, dhi] up to the rounding of
        // fd = (u_c - dlo) * scale (relative 2^-22 of the range), and u_c is
        // within r 2^-20 of r sin(phi_h - phi0); so the sine lies in
        // [dlo/r, dhi/r] widened by 1e-5 plus 2^-18 (2|dlo| + 2|dhi|)/r, which
        // covers both and the fp32 rounding of the ends.
        uint2 out = make_uint2(kAllTiles, 0u);
        if (r_ok) {
            const float m = 1e-5f + 0x1.0p-18f * (2.0f * fabsf(p.dlo) + 2.0f * fabsf(p.dhi)) * inv_r;
            out = arcs(p.dlo * inv_r - m, p.dhi * inv_r + m);
        }
        emit(0, out);
        return;
    }
    if (!p.d0) {
        // 2D (d = 0): the interval below is [-s - m, s + m], s = K r2 / (2r),
        // so one arcsine serves both ends (asin(-v) = -asin(v) up to its
        // error, which the arc widening covers)
        uint2 out = make_uint2(kAllTiles, 0u);
        if (r_ok) {
            const float a = K * r2;
            const float shi = a * half_inv_r + (1e-5f + 0x1.0p-18f * a * inv_r);
            if (isfinite(shi) && (fwd || shi < 1.0f)) {
                const float ahi = arc_asin(fminf(shi, 1.0f));
                const float pm = ph - pi;
                out = make_uint2(tile_range(pack_arc(ph - ahi, ph + ahi, p.n_phi, sc), p),
                                 fwd ? 0u : tile_range(pack_arc(pm - ahi, pm + ahi, p.n_phi, sc), p));
            }
        }
        emit(0, out);
        return;
    }
    for (int l = l_begin; l < l_end; ++l) {
        uint2 out = make_uint2(kAllTiles, 0u);
        const float d = p.d0 ? p.d0[l] : 0.0f;
        const float ad = fabsf(d);
        const float kd = K * ad;
        if (r_ok && ad <= 0x1.0p30f && fabsf(r - ad) >= 0.0301f * (r + ad) && kd <= 0.99f) {
            const float rr = r2 + d * d;
            const float a = K * rr;
            const float b = 2.0f * d;
            const float s1 = (b - a) * half_inv_r * arc_rcp(1.0f - K * d);
            const float s2 = (b + a) * half_inv_r * arc_rcp(1.0f + K * d);
            const float w = arc_rcp(1.0f - kd);
            const float m = 1e-5f + 0x1.0p-18f * (a + 2.0f * ad) * inv_r * w * w;
            out = arcs(fminf(s1, s2) - m, fmaxf(s1, s2) + m);
        }
        if (p.d0 && p.div_fast && fast_div_3d(r, d, ad))
            out.y |= kFastDiv;
        emit(l, out);
    }
}

// Is row j's (cos, sin) the bin centre (j + 1/2) 2 pi / n_phi, within 1e-6 rad
// in angle and 1e-6 in norm (fp64)?  One workgroup; thread 0 writes the flag.
__global__ __launch_bounds__(1024) void table_check_kernel(const float *cos_phi, const float *sin_phi,
                                                           int32_t n_phi, int32_t *ok) {
    const double two_pi = 6.283185307179586;
    int bad = n_phi > 32768 ? 1 : 0;
    for (int j = threadIdx.x; j < n_phi && !bad; j += blockDim.x) {
        const double c = cos_phi[j];
        const double sn = sin_phi[j];
        const double want = (static_cast<double>(j) + 0.5) * two_pi / static_cast<double>(n_phi);
        double diff = fmod(atan2(sn, c) - want, two_pi);
        if (diff > two_pi / 2)
            diff -= two_pi;
        if (diff < -two_pi / 2)
            diff += two_pi;
        const double norm = hypot(c, sn);
        if (!(fabs(diff) < 1e-6) || !(fabs(norm - 1.0) < 1e-6))
            bad = 1;
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0)
        *ok = bad ? 0 : 1;
}

__global__ void prep_kernel(EventState *state, int32_t n_events, unsigned long long *n_votes) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_events) {
        if (state) {
            state[i].key_min = 0xffffffffu;
            state[i].key_max = 0u;
            state[i].n_found = 0;
            state[i].passes = 0;
        }
        if (n_votes)
            n_votes[i] = 0ull;
    }
}

__global__ void prep_batch_kernel(EventState *state, int32_t max_events, const int32_t *n_events_dev,
                                  unsigned long long *n_votes, int32_t *work_counter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < max_events) {
        state[i].key_min = 0xffffffffu;
        state[i].key_max = 0u;
        state[i].n_found = 0;
        state[i].passes = 0;
        if (n_votes && i < *n_events_dev)
            n_votes[i] = 0ull;
    }
    if (i < kQueues && work_counter)
        work_counter[i * kCounterStride] = 0;
}

__global__ void zero_kernel(uint32_t *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0u;
}

using VoteFn = void (*)(VoteArgs);

template <bool U16, bool D3, bool FUSED, bool FWD>
VoteFn pick_shape(int rows, int threads) {
    const int key = rows * 10000 + threads;
    // the forward option comes in the 32-row tiles only (every default shape)
    if constexpr (FWD) {
        switch (key) {
            case 32 * 10000 + 256: return vote_kernel<U16, D3, 32, 256, FUSED, true>;
            case 32 * 10000 + 512: return vote_kernel<U16, D3, 32, 512, FUSED, true>;
            case 32 * 10000 + 1024: return vote_kernel<U16, D3, 32, 1024, FUSED, true>;
            default: return nullptr;
        }
    } else {
        switch (key) {
            case 32 * 10000 + 256: return vote_kernel<U16, D3, 32, 256, FUSED, false>;
            case 32 * 10000 + 512: return vote_kernel<U16, D3, 32, 512, FUSED, false>;
            case 32 * 10000 + 1024: return vote_kernel<U16, D3, 32, 1024, FUSED, false>;
            case 64 * 10000 + 256: return vote_kernel<U16, D3, 64, 256, FUSED, false>;
            case 64 * 10000 + 512: return vote_kernel<U16, D3, 64, 512, FUSED, false>;
            case 64 * 10000 + 1024: return vote_kernel<U16, D3, 64, 1024, FUSED, false>;
            case 128 * 10000 + 256: return vote_kernel<U16, D3, 128, 256, FUSED, false>;
            case 128 * 10000 + 512: return vote_kernel<U16, D3, 128, 512, FUSED, false>;
            case 128 * 10000 + 1024: return vote_kernel<U16, D3, 128, 1024, FUSED, false>;
            default: return nullptr;
        }
    }
}

template <bool FWD>
VoteFn pick_kind(bool u16, bool d3, bool fused, int rows, int threads) {
    if (fused)
        return (!u16 && !d3) ? pick_shape<false, false, true, FWD>(rows, threads) : nullptr;
    if (u16)
        return d3 ? pick_shape<true, true, false, FWD>(rows, threads) : pick_shape<true, false, false, FWD>(rows, threads);
    return d3 ? pick_shape<false, true, false, FWD>(rows, threads) : pick_shape<false, false, false, FWD>(rows, threads);
}

VoteFn pick_vote(bool u16, bool d3, bool fused, bool fwd, int rows, int threads) {
    return fwd ? pick_kind<true>(u16, d3, fused, rows, threads) : pick_kind<false>(u16, d3, fused, rows, threads);
}

hipError_t launch_vote(const VoteArgs &a, bool u16, bool fused, const VoteShape &s, dim3 grid,
                       hipStream_t stream) {
    VoteFn fn = pick_vote(u16, a.g.d0 != nullptr, fused, a.g.forward != 0, s.rows, s.threads);
    if (!fn)
        return hipErrorInvalidValue;
    const size_t lds = vote_lds_bytes(s, a.g.n_kappa);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, grid, dim3(s.threads), lds, stream, a);
    return hipGetLastError();
}

void fill_inputs(VoteArgs &a, const VoteInputs &in) {
    a.hits = in.hits;
    a.ranges = in.ranges;
    a.range_stride = in.range_stride;
    a.range_step = in.range_step;
    a.mask_mode = in.mask_mode;
}

void set_geometry(VoteArgs &a, const GridArgs &g, const VoteShape &s, bool fused) {
    const TileGeom tg = vote_tile_geom(g, s, fused);
    a.tiles_per_slice = tg.tiles;
    a.tile_stride = tg.stride;
    a.tile_off = tg.halo ? -1 : 0;
}

}  // namespace

TileGeom vote_tile_geom(const GridArgs &g, const VoteShape &s, bool fused) {
    TileGeom tg{};
    tg.stride = fused ? s.rows - 2 : s.rows;
    tg.halo = fused ? 1 : 0;
    tg.tiles = (g.n_phi + tg.stride - 1) / tg.stride;
    return tg;
}

size_t vote_lds_bytes(const VoteShape &s, int32_t n_kappa) {
    // kappa-major int32 tile: n_kappa columns of `rows` dwords, plus the spare column
    return (static_cast<size_t>(n_kappa) + 1) * static_cast<size_t>(s.rows) * sizeof(uint32_t);
}

int32_t vote_groups_per_cu(const VoteShape &s, int32_t n_kappa) {
    // workgroups of shape s resident on one CU: LDS (in 1 KiB granules, the
    // dynamic tile plus the static scratch) and 32 wavefronts per CU
    const size_t st = s.threads <= 256 ? sizeof(TileScratch<256>)
                      : s.threads <= 512 ? sizeof(TileScratch<512>) : sizeof(TileScratch<1024>);
    const size_t lds = (vote_lds_bytes(s, n_kappa) + st + 1023) / 1024 * 1024;
    const int by_lds = static_cast<int>((160u * 1024u) / lds);
    const int by_waves = 32 / std::max(1, s.threads / 64);
    return std::max(1, std::min(by_lds, by_waves));
}

bool vote_shape_supported(const VoteShape &s, bool u16, int32_t n_kappa, bool forward) {
    if (!pick_vote(u16, false, false, forward, s.rows, s.threads))
        return false;
    if (s.split < 1 || s.split > 64)
        return false;
    // dynamic tile + static scratch (staged hits, compaction and reductions)
    return vote_lds_bytes(s, n_kappa) + sizeof(TileScratch<1024>) <= 160u * 1024u;
}

bool vote_near_band(const GridArgs &g, float *band, float *off) {
    // Bound chain on |kf| <= K = n_kappa + 2, with u = 2^-24 (one rounding per
    // operation), M = |kappa_min| kappa_scale, kf_r the bin in real arithmetic
    // of the same fp32 operands and P its slope term, |P| <= K + M:
    //   exact kf:  |kf - kf_r| <= u |P| (the quotient) + 2u |kf_r| (two roundings after it);
    //   kf1:       |kf1 - (kf_r + E)| <= 3u |P| (the reciprocal's 1 ulp, the product's
    //              rounding) + u (E + M) (off) + u |kf1| (the FMA), |kf1| <= K + 1;
    // second-order terms fit in the factor 1 + 2^-20.  A lane outside the band
    // [k, k + 2E) decides alike whenever E exceeds the sum (|kf1 - (kf + E)|
    // < E, vote_math.h); E is the sum plus a quarter of margin.
    // Beyond the band (|kf_r| > K) the same relative bounds keep kf and kf1 out
    // of [0, n_kappa) while K + M <= 2^20.  kappa_scale in [2^-60, 2^60] keeps
    // the 2D hit constant w = RN(y kappa_scale) normal and finite.
    const double ks = g.kappa_scale;
    const double km = std::fabs(static_cast<double>(g.kappa_min));
    if (!(ks >= 0x1.0p-60 && ks <= 0x1.0p60) || !std::isfinite(km))
        return false;
    const double K = static_cast<double>(g.n_kappa) + 2.0;
    const double M = km * ks;
    if (!(K + M <= 0x1.0p20))
        return false;
    const double u = 0x1.0p-24;
    const double ekf = (4.0 * u * (K + M) + 2.0 * u * K + u * (1.0 + M) + u * (K + 1.0)) * (1.0 + 0x1.0p-20);
    const double E = 1.25 * ekf;
    if (!(E <= 1.0 / 64.0))
        return false;
    float b = static_cast<float>(2.0 * E);
    if (static_cast<double>(b) < 2.0 * E)
        b = std::nextafter(b, INFINITY);
    *band = b;
    *off = static_cast<float>(E - static_cast<double>(g.kappa_min) * ks);
    return true;
}

int32_t vote_tiles_per_slice(const GridArgs &g, const VoteShape &s, bool fused) {
    return vote_tile_geom(g, s, fused).tiles;
}

int32_t fused_chunk_cap(const GridArgs &g, const VoteShape &s) {
    // Survivors of S interior rows: an independent set of the king's graph.
    const int32_t S = s.rows - 2;
    return ((S + 1) / 2) * ((g.n_kappa + 1) / 2);
}

hipError_t launch_hit_prep(const GridArgs &g, const TileGeom &tg, const float *x, const float *y, int64_t n_hits,
                           const int64_t *n_hits_dev, float4 *hits, uint2 *ranges, int64_t range_stride,
                           bool div_fast, bool masks, const int32_t *table_ok, hipStream_t stream) {
    if (n_hits <= 0)
        return hipSuccess;
    PrepArgs p{};
    p.x = x;
    p.y = y;
    p.n_hits = n_hits;
    p.n_hits_dev = n_hits_dev;
    p.hits = hits;
    p.ranges = ranges;
    p.range_stride = range_stride;
    p.d0 = g.d0;
    p.n_phi = g.n_phi;
    p.n_d0 = g.n_d0;
    p.tiles = tg.tiles;
    p.tile_stride = tg.stride;
    p.halo = tg.halo;
    p.div_fast = div_fast ? 1 : 0;
    p.w_scale = g.near_band > 0.0f ? g.kappa_scale : 1.0f;
    p.mask_mode = masks && ranges && tg.tiles <= kMaskTiles ? 1 : 0;
    p.table_ok = table_ok;
    const double kmin = g.kappa_min;
    const double kmax = static_cast<double>(g.kappa_min) + static_cast<double>(g.n_kappa) / g.kappa_scale;
    const double K = fmax(fabs(kmin), fabs(kmax)) * (1.0 + 1e-3);
    float Kf = static_cast<float>(K);
    if (static_cast<double>(Kf) < K)
        Kf = nextafterf(Kf, INFINITY);
    p.kabs = std::isnan(K) ? INFINITY : Kf;
    p.straight = g.straight;
    p.forward = g.forward;
    if (g.straight) {
        const double lo = g.kappa_min;
        const double hi = lo + static_cast<double>(g.n_kappa) / g.kappa_scale;
        float flo = static_cast<float>(lo), fhi = static_cast<float>(hi);
        if (static_cast<double>(flo) > lo)
            flo = nextafterf(flo, -INFINITY);
        if (static_cast<double>(fhi) < hi)
            fhi = nextafterf(fhi, INFINITY);
        p.dlo = std::isfinite(flo) ? flo : -INFINITY;
        p.dhi = std::isfinite(fhi) ? fhi : INFINITY;
    }
    p.stride_magic = tg.stride > 1
        ? static_cast<uint32_t>(((1ull << 32) + static_cast<uint64_t>(tg.stride) - 1) / static_cast<uint64_t>(tg.stride))
        : 0u;
    const unsigned blocks = static_cast<unsigned>((n_hits + 255) / 256);
    const unsigned groups = ranges ? static_cast<unsigned>((g.n_d0 + kPrepSlices - 1) / kPrepSlices) : 1u;
    hipLaunchKernelGGL(hit_prep_kernel, dim3(blocks, groups), dim3(256), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_table_check(const float *cos_phi, const float *sin_phi, int32_t n_phi, int32_t *ok,
                              hipStream_t stream) {
    hipLaunchKernelGGL(table_check_kernel, dim3(1), dim3(1024), 0, stream, cos_phi, sin_phi, n_phi, ok);
    return hipGetLastError();
}

hipError_t launch_prep(EventState *state, int32_t n_events, unsigned long long *n_votes,
                       hipStream_t stream) {
    const int blocks = (n_events + 255) / 256;
    hipLaunchKernelGGL(prep_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream, state, n_events, n_votes);
    return hipGetLastError();
}

hipError_t launch_prep_batch(EventState *state, int32_t max_events, const int32_t *n_events_dev,
                             unsigned long long *n_votes, int32_t *work_counter, hipStream_t stream) {
    const int blocks = (max_events + 255) / 256;
    hipLaunchKernelGGL(prep_batch_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream, state, max_events,
                       n_events_dev, n_votes, work_counter);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t *p, int64_t n_dwords, hipStream_t stream) {
    if (n_dwords <= 0)
        return hipSuccess;
    int64_t blocks = (n_dwords + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, p, n_dwords);
    return hipGetLastError();
}

hipError_t launch_vote_single(const GridArgs &g, bool u16, const VoteShape &s, const VoteInputs &in,
                              int32_t n_hits, uint32_t *acc, unsigned long long *n_votes, hipStream_t stream,
                              unsigned long long *pairs) {
    VoteArgs a{};
    a.pairs = pairs;
    a.g = g;
    fill_inputs(a, in);
    a.n_hits = n_hits;
    a.split = s.split;
    set_geometry(a, g, s, false);
    a.acc = acc;
    a.n_votes = n_votes;
    hipError_t e = hipSuccess;
    if (s.split > 1)
        e = launch_zero(acc, g.acc_dwords, stream);
    if (e != hipSuccess)
        return e;
    dim3 grid(static_cast<unsigned>(a.tiles_per_slice * vote_slice_units(g, u16)), static_cast<unsigned>(s.split));
    return launch_vote(a, u16, false, s, grid, stream);
}

hipError_t launch_vote_batch(const GridArgs &g, bool u16, bool fused, const VoteShape &s, const VoteInputs &in,
                             const EventDesc *desc, const QueueDesc *queues, const WorkItem *items,
                             int32_t max_items, int32_t *work_counter, int32_t persistent_groups, uint32_t *acc,
                             unsigned long long *n_votes, const SortWork *w, int32_t threshold,
                             hipStream_t stream, unsigned long long *pairs) {
    VoteArgs a{};
    a.pairs = pairs;
    a.g = g;
    fill_inputs(a, in);
    a.split = 1;
    set_geometry(a, g, s, fused);
    a.desc = desc;
    a.items = items;
    a.queues = queues;
    a.acc = acc;
    a.n_votes = n_votes;
    if (w)
        a.w = *w;
    a.threshold = threshold;
    unsigned blocks = static_cast<unsigned>(max_items);
    if (work_counter && persistent_groups > 0) {
        a.work_counter = work_counter;
        blocks = static_cast<unsigned>(persistent_groups < max_items ? persistent_groups : max_items);
    }
    if (blocks == 0)
        return hipSuccess;
    return launch_vote(a, u16, fused, s, dim3(blocks), stream);
}

}  // namespace hough
