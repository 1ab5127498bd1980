// Hough vote kernels for gfx950.
//
// Section 3: every hypothesis starts with zero votes and every hit adds one
// vote to each hypothesis it lies on; Section 4: the work for each hit is
// independent of the others.
//
// Layout.  The accumulator of one d0 slice is cut into tiles of 64 (or 128)
// consecutive phi0 rows.  A workgroup owns one tile as a private LDS
// accumulator; each lane owns one phi0 row (two for 128-row tiles) and keeps
// that row's cos/sin and the slice's d0 in registers; each wavefront takes
// one hit at a time (hit data are wave-uniform), so a wavefront evaluates 64
// rows of a hit per instruction.  The finished tile is flushed to HBM with
// coalesced stores -- no global atomics on the accumulator -- and the vote
// count is reduced per wavefront and added once per workgroup.
//
// Culling.  A hit can only vote in the phi0 rows where its curvature lies in
// the kappa range, which is two arcs of phi0 per d0 slice.  hit_prep_kernel
// computes, per hit and d0 slice, a conservative bit mask of the tiles those
// arcs touch (widened by bounds on every fp32 rounding of the vote
// arithmetic, see below); the vote loop skips a hit for a tile whose bit is
// clear.  Which votes are cast is still decided only by the exact fp32 test,
// so culling changes no result.
//
// Arithmetic is the fp32 definition in hough.h, op for op; this file is
// compiled with -ffp-contract=off and the default correctly rounded divide.
// r2 = x*x + y*y is computed with the same operations when a hit is staged.  For the 2D grid (d0 == +0) the numerator 2*(u - 0) equals 2*u
// and the denominator (r2 - 0*u) + 0*0 equals r2 for every finite u, and both
// forms give NaN or an out-of-range kf otherwise, so the 2D kernels use
// 2*u / r2.
//
// uint16 accumulators are packed two cells per dword in LDS (even kappa bin in
// the low half): a vote adds 1 or 0x10000 with one 32-bit LDS atomic.  The low
// half can never carry into the high half because a cell receives at most one
// vote per hit and u16 events hold at most 65535 hits.
//
// Fused peak search (2D int32 batches).  Tiles then overlap by two rows: a
// tile votes S interior rows plus one halo row on each side, finds the local
// maxima of its interior rows straight from LDS and appends them in cell
// order to its staging list; the accumulator need not reach HBM at all.
#pragma clang fp contract(off)

#include "hough_impl.h"
#include "peak_tile.h"

namespace hough {
namespace {

struct VoteArgs {
    GridArgs g;
    const float *x;
    const float *y;
    const uint32_t *mask;       // [n_d0][mask_stride] tile masks; or one all-ones word (step 0)
    int64_t mask_stride;
    int32_t mask_step;          // 1 with masks, 0 without
    int32_t n_hits;             // single event
    int32_t split;              // single event: hit chunks per tile
    int32_t tiles_per_slice;
    int32_t tile_stride;        // tile t starts at row t*tile_stride + tile_off
    int32_t tile_off;           // 0, or -1 for fused tiles
    int32_t lds_stride;         // dwords per LDS row
    const EventDesc *desc;      // batch: per-event hit ranges
    const WorkItem *items;      // batch: tile list, or nullptr for a single event
    const int32_t *n_items;     // batch: live item count (device)
    int32_t *work_counter;      // batch, persistent: next item to take
    uint32_t *acc;              // dwords; fused batches may pass nullptr
    unsigned long long *n_votes;
    SortWork w;                 // fused: staging lists
    int32_t threshold;          // fused
};

constexpr int kHitBlock = 1024;   // hits staged in LDS per round

template <int NT>
struct TileScratch {
    float4 hits[kHitBlock];         // kept hits of the current block: x, y, r2
    CompactScratch<NT> sc;
    unsigned long long red[NT / 64];
    int32_t n_kept[2];
    int32_t next_item;
};

__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <bool U16>
__device__ __forceinline__ uint32_t cell_sum(uint32_t v) {
    return U16 ? (v & 0xffffu) + (v >> 16) : v;
}

// Vote hits [h_begin, h_end) of event e into tile t of d0 slice l, then either
// flush it (unfused) or search its interior rows for peaks (fused).
template <bool U16, bool D3, int RPT, int NT, bool FUSED>
__device__ void vote_tile(const VoteArgs &a, int e, int l, int t, int64_t h_begin, int64_t h_end,
                          uint32_t *__restrict__ acc_event, bool atomic_flush, unsigned long long *n_votes,
                          uint32_t *lds, TileScratch<NT> &ts) {
    constexpr int R = 64 * RPT;
    constexpr int NW = NT / 64;
    const GridArgs &g = a.g;
    const int tid = threadIdx.x;
    const int stride = a.lds_stride;
    const int n_phi = g.n_phi;
    const int first = t * a.tile_stride + a.tile_off;      // may be -1 for a fused tile
    int len, s_here = 0;
    if constexpr (FUSED) {
        s_here = min(a.tile_stride, n_phi - t * a.tile_stride);
        len = s_here + 2;
    } else {
        len = min(R, n_phi - first);
    }

    for (int i = tid; i < len * stride; i += NT)
        lds[i] = 0u;
    if constexpr (FUSED) {
        for (int i = tid; i < kDigits; i += NT)
            ts.sc.hist[i] = 0u;
    }
    __syncthreads();

    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    float c[RPT], s[RPT];
    int rowoff[RPT];
    bool live[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = lane + 64 * i;
        live[i] = r < len;
        int j = first + r;
        if (j < 0)
            j += n_phi;
        if (j >= n_phi)
            j -= n_phi;
        if (!live[i])
            j = 0;
        c[i] = g.cos_phi[j];
        s[i] = g.sin_phi[j];
        rowoff[i] = r * stride;
    }
    const float d = D3 ? g.d0[l] : 0.0f;
    // Let the row constants land now: the memory counter is in order, so a
    // first use inside the hit loop would also wait for the hit prefetches.
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
    const float d2 = 2.0f * d;
    const float dd = d * d;
    const float kmin = g.kappa_min;
    const float kscale = g.kappa_scale;
    const float nkf = static_cast<float>(g.n_kappa);
    const float *__restrict__ xs = a.x;
    const float *__restrict__ ys = a.y;
    const uint32_t *__restrict__ mrow = a.mask + static_cast<int64_t>(l) * a.mask_stride;
    const int64_t mstep = a.mask_step;
    const uint32_t tbit = 1u << (t & 31);

    // One evaluation: hit (xh, yh, r2) at this lane's row i.
    auto eval = [&](float xh, float yh, float r2) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const float u = yh * c[i] - xh * s[i];
            float kappa;
            if constexpr (D3) {
                const float num = 2.0f * (u - d);
                const float den = (r2 - d2 * u) + dd;
                kappa = num / den;
            } else {
                kappa = (2.0f * u) / r2;
            }
            const float kf = (kappa - kmin) * kscale;
            if (live[i] && kf >= 0.0f && kf < nkf) {
                const int k = static_cast<int>(kf);
                if constexpr (U16)
                    lds_add(&lds[rowoff[i] + (k >> 1)], (k & 1) ? 0x10000u : 1u);
                else
                    lds_add(&lds[rowoff[i] + k], 1u);
            }
        }
    };

    // Hits stream through LDS in blocks of kHitBlock: every thread loads
    // kHitBlock/NT hits (the loads for the next block are in flight while the
    // current one is evaluated), keeps those whose tile bit is set, and the
    // kept hits are packed as (x, y, r2) for wave-uniform LDS reads.
    constexpr int PER = kHitBlock / NT;
    float px[PER], py[PER];
    uint32_t pm[PER];
    // All loads of a block are issued back to back and unconditionally (the
    // index is clamped), so they stay in flight during the previous block's
    // evaluation; whether a hit is kept is decided when it is staged.
    auto fetch = [&](int64_t b0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int64_t h = min(b0 + q * NT + tid, h_end - 1);
            pm[q] = mrow[h * mstep];
            px[q] = xs[h];
            py[q] = ys[h];
        }
    };
    if (h_begin < h_end)
        fetch(h_begin);
    int parity = 0;
    if (tid == 0) {
        ts.n_kept[0] = 0;
        ts.n_kept[1] = 0;
    }
    for (int64_t b0 = h_begin; b0 < h_end; b0 += kHitBlock, parity ^= 1) {
        __syncthreads();                         // the previous block is fully evaluated
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const bool keep = b0 + q * NT + tid < h_end && (pm[q] & tbit);
            const uint64_t m = __ballot(keep);
            int base = 0;
            if (lane == 0 && m)
                base = atomicAdd(&ts.n_kept[parity], __popcll(m));
            base = __shfl(base, 0, 64);
            if (keep)
                ts.hits[base + rank_below(m)] = make_float4(px[q], py[q], px[q] * px[q] + py[q] * py[q], 0.0f);
        }
        __syncthreads();
        const int n = ts.n_kept[parity];
        if (tid == 0)
            ts.n_kept[parity ^ 1] = 0;           // free since every thread passed the last barrier
        if (b0 + kHitBlock < h_end)
            fetch(b0 + kHitBlock);
        int i = wave;
        for (; i + NW < n; i += 2 * NW) {
            const float4 h0 = ts.hits[i];
            const float4 h1 = ts.hits[i + NW];
            eval(h0.x, h0.y, h0.z);
            eval(h1.x, h1.y, h1.z);
        }
        if (i < n) {
            const float4 h0 = ts.hits[i];
            eval(h0.x, h0.y, h0.z);
        }
    }
    __syncthreads();

    const int rd = g.row_dwords;
    unsigned long long votes = 0;
    if constexpr (FUSED) {
        // Interior rows 1..s_here of the tile are phi0 rows j_first.. of slice 0.
        const int j_first = t * a.tile_stride;
        const int nk = g.n_kappa;
        const int32_t *tile = reinterpret_cast<const int32_t *>(lds);
        const int32_t thr = a.threshold;
        Cand *out = a.w.s0.stage + (static_cast<int64_t>(e) * a.w.s0.n_blocks0 + t) * a.w.s0.cap0;
        uint32_t kmin_key, kmax_key;
        const int count = compact_ordered<NT>(
            s_here * nk,
            [&](int idx, int32_t *v, int32_t *cell) {
                const int rr = idx / nk;
                const int k = idx - rr * nk;
                const int32_t *row = tile + (rr + 1) * stride;
                const int32_t val = row[k];
                if (val < thr || !is_peak_2d(row, stride, nk, k, val))
                    return false;
                *v = val;
                *cell = (j_first + rr) * nk + k;
                return true;
            },
            out, ts.sc, &kmin_key, &kmax_key);
        publish_block<NT>(a.w, e, t, count, ts.sc, kmin_key, kmax_key);
        uint32_t *dst = acc_event ? acc_event + static_cast<int64_t>(j_first) * rd : nullptr;
        for (int rr = 0; rr < s_here; ++rr)
            for (int wd = tid; wd < rd; wd += NT) {
                const uint32_t v = lds[(rr + 1) * stride + wd];
                votes += v;
                if (dst)
                    dst[static_cast<int64_t>(rr) * rd + wd] = v;
            }
    } else {
        uint32_t *dst = acc_event + (static_cast<int64_t>(l) * n_phi + first) * rd;
        for (int rr = 0; rr < len; ++rr)
            for (int wd = tid; wd < rd; wd += NT) {
                const uint32_t v = lds[rr * stride + wd];
                votes += cell_sum<U16>(v);
                if (!atomic_flush)
                    dst[static_cast<int64_t>(rr) * rd + wd] = v;
                else if (v)
                    atomicAdd(&dst[static_cast<int64_t>(rr) * rd + wd], v);
            }
    }
    if (n_votes) {
        const unsigned long long wsum = wave_sum_u64(votes);
        if (lane == 0)
            ts.red[wave] = wsum;
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int wv = 0; wv < NW; ++wv)
                tot += ts.red[wv];
            if (tot)
                atomicAdd(n_votes, tot);
        }
    }
    __syncthreads();   // the LDS tile and scratch are reused by the next item
}

template <bool U16, bool D3, int RPT, int NT, bool FUSED>
__global__ __launch_bounds__(NT) void vote_kernel(VoteArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ TileScratch<NT> ts;
    const int T = a.tiles_per_slice;

    if (a.items == nullptr) {
        const int tile = blockIdx.x;
        const int l = tile / T;
        const int t = tile - l * T;
        const int64_t n = a.n_hits;
        const int64_t per = (n + a.split - 1) / a.split;
        const int64_t hb = static_cast<int64_t>(blockIdx.y) * per;
        const int64_t he = min(n, hb + per);
        vote_tile<U16, D3, RPT, NT, FUSED>(a, 0, l, t, hb, he, a.acc, a.split > 1, a.n_votes, lds, ts);
        return;
    }
    const int32_t n_items = *a.n_items;
    int32_t it = blockIdx.x;
    for (;;) {
        if (a.work_counter) {
            if (threadIdx.x == 0)
                ts.next_item = atomicAdd(a.work_counter, 1);
            __syncthreads();
            it = ts.next_item;
            __syncthreads();
        }
        if (it >= n_items)
            return;
        const WorkItem wi = a.items[it];
        const EventDesc ev = a.desc[wi.event];
        const int l = wi.tile / T;
        const int t = wi.tile - l * T;
        uint32_t *acc_e = a.acc ? a.acc + static_cast<int64_t>(wi.event) * a.g.acc_dwords : nullptr;
        vote_tile<U16, D3, RPT, NT, FUSED>(a, wi.event, l, t, ev.hit_begin, ev.hit_end, acc_e, false,
                                           a.n_votes ? a.n_votes + wi.event : nullptr, lds, ts);
        if (!a.work_counter)
            return;
    }
}

// ---------------------------------------------------------------------------
// Per-hit preparation: r2 and conservative tile masks.
//
// Bound used for the masks (all angles in radians, K = max |kappa edge|).
// If a vote is cast, the fp32 curvature kappa_c lies within K(1 + 2^-19).
// kappa_c rounds num_c / den_c, where num_c = 2(u_c - d) to 2^-24 relative,
// u_c = y c - x s to r 2^-20 absolute (fp32 products, and fp32 cos/sin of the
// bin centre), and den_c equals r^2 - 2 d u_c + d^2 to 2^-21 (r + |d|)^2
// absolute.  When |r - |d|| >= 0.1 (r + |d|) the exact denominator is at least
// (r - |d|)^2, so kappa(u_c) = 2(u_c - d)/(r^2 + d^2 - 2 d u_c) is within
// relative 5e-5 of kappa_c and |kappa(u_c)| <= K' = K (1 + 1e-3).  kappa(u) is
// monotone in u, so u_c lies between u(-K') and u(K') with
// u(k) = (k (r^2 + d^2) + 2 d) / (2 (1 + k d)), and r sin(phi_h - phi0) lies
// in that interval widened by r 1e-5.  The two phi0 arcs that satisfy this,
// widened by 1e-5 rad and one row on each side, give the rows (and tiles)
// that can receive the hit's votes.  Hits that are not finite, sit within
// 1e-15 of the origin or beyond 1e15, or fail the conditioning test keep
// every tile.  The phi0 table must hold the bin centres (j + 1/2) 2 pi / n_phi
// (checked when the context is created; otherwise culling stays off).
// ---------------------------------------------------------------------------

struct PrepArgs {
    const float *x;
    const float *y;
    int64_t n_hits;
    const int64_t *n_hits_dev;  // batch: live hit count (overrides n_hits), or nullptr
    uint32_t *mask;
    int64_t mask_stride;
    const float *d0;            // nullptr for 2D
    int32_t n_phi;
    double kabs;
    int32_t tiles;
    int32_t tile_stride;
    int32_t tile_off;
    int32_t tile_rows;          // rows a tile votes, halo included
};

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
    const int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

__device__ __forceinline__ uint32_t bit_range(int64_t lo, int64_t hi) {
    const int64_t n = hi - lo + 1;
    const uint32_t ones = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
    return ones << lo;
}

// Tiles whose rows meet the unwrapped row range [jlo, jhi].
__device__ uint32_t tiles_meeting(const PrepArgs &p, int64_t jlo, int64_t jhi, uint32_t all) {
    const int64_t n = p.n_phi;
    if (jhi < jlo)
        return 0u;
    if (jhi - jlo + 1 >= n)
        return all;
    const int64_t sh = floor_div(jlo, n) * n;
    jlo -= sh;
    jhi -= sh;
    const int64_t pieces[2][2] = {{jlo, jhi < n ? jhi : n - 1}, {0, jhi - n}};
    const int n_pieces = jhi >= n ? 2 : 1;
    uint32_t m = 0u;
    for (int q = 0; q < n_pieces; ++q) {
        for (int img = -1; img <= 1; ++img) {
            const int64_t lo = pieces[q][0] - img * n - p.tile_off;
            const int64_t hi = pieces[q][1] - img * n - p.tile_off;
            int64_t tlo = -floor_div(-(lo - p.tile_rows + 1), p.tile_stride);   // ceil
            int64_t thi = floor_div(hi, p.tile_stride);
            if (tlo < 0)
                tlo = 0;
            if (thi > p.tiles - 1)
                thi = p.tiles - 1;
            if (tlo <= thi)
                m |= bit_range(tlo, thi);
        }
    }
    return m & all;
}

__device__ uint32_t arc_tiles(const PrepArgs &p, double phi_a, double phi_b, uint32_t all) {
    const double dphi = 6.283185307179586 / p.n_phi;
    const double tol = 1e-5;
    const int64_t jlo = static_cast<int64_t>(ceil((phi_a - tol) / dphi - 0.5)) - 1;
    const int64_t jhi = static_cast<int64_t>(floor((phi_b + tol) / dphi - 0.5)) + 1;
    return tiles_meeting(p, jlo, jhi, all);
}

__global__ void hit_prep_kernel(PrepArgs p) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    const int64_t n = p.n_hits_dev ? *p.n_hits_dev : p.n_hits;
    if (i >= n)
        return;
    const float x = p.x[i];
    const float y = p.y[i];
    const uint32_t all = p.tiles >= 32 ? 0xffffffffu : ((1u << p.tiles) - 1u);
    uint32_t m = all;
    const double X = x, Y = y;
    const double r = sqrt(X * X + Y * Y);
    const double d = p.d0 ? static_cast<double>(p.d0[l]) : 0.0;
    const double ad = fabs(d);
    const double K = p.kabs * (1.0 + 1e-3);
    const bool finite_in = isfinite(X) && isfinite(Y) && isfinite(d);
    if (finite_in && r > 1e-15 && r < 1e15 && ad < 1e15 && fabs(r - ad) >= 0.1 * (r + ad) && K * ad < 0.5) {
        const double rr = r * r + d * d;
        const double u1 = (-K * rr + 2.0 * d) / (2.0 * (1.0 - K * d));
        const double u2 = (K * rr + 2.0 * d) / (2.0 * (1.0 + K * d));
        const double slo = (fmin(u1, u2) - r * 1e-5) / r;
        const double shi = (fmax(u1, u2) + r * 1e-5) / r;
        if (slo > 1.0 || shi < -1.0) {
            m = 0u;
        } else if (!(slo <= -1.0 && shi >= 1.0)) {
            const double alo = asin(fmax(slo, -1.0));
            const double ahi = asin(fmin(shi, 1.0));
            const double ph = atan2(Y, X);
            const double pi = 3.141592653589793;
            m = arc_tiles(p, ph - ahi, ph - alo, all) | arc_tiles(p, ph - pi + alo, ph - pi + ahi, all);
        }
    }
    p.mask[static_cast<int64_t>(l) * p.mask_stride + i] = m;
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
    if (i == 0 && work_counter)
        *work_counter = 0;
}

__global__ void zero_kernel(uint32_t *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0u;
}

using VoteFn = void (*)(VoteArgs);

template <bool U16, bool D3, bool FUSED>
VoteFn pick_shape(int rows, int threads) {
    const int key = rows * 10000 + threads;
    switch (key) {
        case 64 * 10000 + 256: return vote_kernel<U16, D3, 1, 256, FUSED>;
        case 64 * 10000 + 512: return vote_kernel<U16, D3, 1, 512, FUSED>;
        case 64 * 10000 + 1024: return vote_kernel<U16, D3, 1, 1024, FUSED>;
        case 128 * 10000 + 256: return vote_kernel<U16, D3, 2, 256, FUSED>;
        case 128 * 10000 + 512: return vote_kernel<U16, D3, 2, 512, FUSED>;
        case 128 * 10000 + 1024: return vote_kernel<U16, D3, 2, 1024, FUSED>;
        default: return nullptr;
    }
}

VoteFn pick_vote(bool u16, bool d3, bool fused, int rows, int threads) {
    if (fused)
        return (!u16 && !d3) ? pick_shape<false, false, true>(rows, threads) : nullptr;
    if (u16)
        return d3 ? pick_shape<true, true, false>(rows, threads) : pick_shape<true, false, false>(rows, threads);
    return d3 ? pick_shape<false, true, false>(rows, threads) : pick_shape<false, false, false>(rows, threads);
}

hipError_t launch_vote(const VoteArgs &a, bool u16, bool fused, const VoteShape &s, dim3 grid,
                       hipStream_t stream) {
    VoteFn fn = pick_vote(u16, a.g.d0 != nullptr, fused, s.rows, s.threads);
    if (!fn)
        return hipErrorInvalidValue;
    const size_t lds = vote_lds_bytes(s, a.g.row_dwords);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, grid, dim3(s.threads), lds, stream, a);
    return hipGetLastError();
}

void tile_geometry(const GridArgs &g, const VoteShape &s, bool fused, int32_t *tiles, int32_t *stride,
                   int32_t *off) {
    if (fused) {
        *stride = s.rows - 2;
        *off = -1;
    } else {
        *stride = s.rows;
        *off = 0;
    }
    *tiles = (g.n_phi + *stride - 1) / *stride;
}

}  // namespace

size_t vote_lds_bytes(const VoteShape &s, int32_t row_dwords) {
    return static_cast<size_t>(s.rows) * static_cast<size_t>(row_dwords + s.pad) * sizeof(uint32_t);
}

bool vote_shape_supported(const VoteShape &s, bool u16, int32_t row_dwords) {
    if (!pick_vote(u16, false, false, s.rows, s.threads))
        return false;
    if (s.pad < 0 || s.pad > 1 || s.split < 1 || s.split > 64)
        return false;
    // dynamic tile + static scratch (staged hits, compaction and reductions)
    return vote_lds_bytes(s, row_dwords) + sizeof(TileScratch<1024>) <= 160u * 1024u;
}

int32_t vote_tiles_per_slice(const GridArgs &g, const VoteShape &s, bool fused) {
    int32_t tiles, stride, off;
    tile_geometry(g, s, fused, &tiles, &stride, &off);
    return tiles;
}

int32_t fused_chunk_cap(const GridArgs &g, const VoteShape &s) {
    // Survivors of S interior rows: an independent set of the king's graph.
    const int32_t S = s.rows - 2;
    return ((S + 1) / 2) * ((g.n_kappa + 1) / 2);
}

hipError_t launch_hit_prep(const GridArgs &g, const VoteShape &s, bool fused, const float *x, const float *y,
                           int64_t n_hits, const int64_t *n_hits_dev, uint32_t *mask, int64_t mask_stride,
                           hipStream_t stream) {
    if (n_hits <= 0)
        return hipSuccess;
    PrepArgs p{};
    p.x = x;
    p.y = y;
    p.n_hits = n_hits;
    p.n_hits_dev = n_hits_dev;
    p.mask = mask;
    p.mask_stride = mask_stride;
    p.d0 = g.d0;
    p.n_phi = g.n_phi;
    const double kmin = g.kappa_min;
    const double kmax = static_cast<double>(g.kappa_min) + static_cast<double>(g.n_kappa) / g.kappa_scale;
    p.kabs = fmax(fabs(kmin), fabs(kmax));
    tile_geometry(g, s, fused, &p.tiles, &p.tile_stride, &p.tile_off);
    p.tile_rows = fused ? p.tile_stride + 2 : s.rows;
    const unsigned blocks = static_cast<unsigned>((n_hits + 255) / 256);
    hipLaunchKernelGGL(hit_prep_kernel, dim3(blocks, g.n_d0), dim3(256), 0, stream, p);
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
                              int32_t n_hits, uint32_t *acc, unsigned long long *n_votes, hipStream_t stream) {
    VoteArgs a{};
    a.g = g;
    a.x = in.x;
    a.y = in.y;
    a.mask = in.mask;
    a.mask_stride = in.mask_stride;
    a.mask_step = in.mask_step;
    a.n_hits = n_hits;
    a.split = s.split;
    tile_geometry(g, s, false, &a.tiles_per_slice, &a.tile_stride, &a.tile_off);
    a.lds_stride = g.row_dwords + s.pad;
    a.acc = acc;
    a.n_votes = n_votes;
    hipError_t e = hipSuccess;
    if (s.split > 1)
        e = launch_zero(acc, g.acc_dwords, stream);
    if (e != hipSuccess)
        return e;
    dim3 grid(static_cast<unsigned>(a.tiles_per_slice * g.n_d0), static_cast<unsigned>(s.split));
    return launch_vote(a, u16, false, s, grid, stream);
}

hipError_t launch_vote_batch(const GridArgs &g, bool u16, bool fused, const VoteShape &s, const VoteInputs &in,
                             const EventDesc *desc, const int32_t *n_items_dev, const WorkItem *items,
                             int32_t max_items, int32_t *work_counter, int32_t persistent_groups, uint32_t *acc,
                             unsigned long long *n_votes, const SortWork *w, int32_t threshold,
                             hipStream_t stream) {
    VoteArgs a{};
    a.g = g;
    a.x = in.x;
    a.y = in.y;
    a.mask = in.mask;
    a.mask_stride = in.mask_stride;
    a.mask_step = in.mask_step;
    a.split = 1;
    tile_geometry(g, s, fused, &a.tiles_per_slice, &a.tile_stride, &a.tile_off);
    a.lds_stride = g.row_dwords + s.pad;
    a.desc = desc;
    a.items = items;
    a.n_items = n_items_dev;
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
