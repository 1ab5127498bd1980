// Hit association: the hits that make each track candidate (Section 3: a
// candidate is a local maximum of the votes cast by the hits compatible with
// it).  Hit h belongs to candidate C = (lc, jc, kc) when h votes into a cell
// of C's window (lc + dl, jc + dj, kc + dk), dl, dj, dk in {-1, 0, 1}: phi0
// modulo n_phi, d0 and kappa inside the grid -- the window of the peak rule.
//
// The vote is recomputed here with the grid's family and forward option: in
// its plain binary32 form, operation for operation the definition in hough.h
// (this file is compiled with -ffp-contract=off; the division is the
// correctly rounded operator, the range test the compare form), or -- for
// prompt 2D grids with a phi0 table of bin centres -- as the vote kernels do
// it, an approximate bin from one FMA and that exact form wherever the
// estimate cannot decide (vote_math.h), which gives the same bins.
//
// Layout: the context's cell map holds, per cell, 1 + the index of the
// candidate there (0: none), and a bitmap of the cells that hold one: per
// (d0, phi0) row, bit kc + 1 of assoc_row_words(n_kappa) dwords (about 1 MB
// for the displaced grid, so it stays in L2).
//
// Work: hits are first put in azimuth order (a counting sort into the
// context's hit records), so that the lanes of a wavefront are hits of
// similar direction, whose votes fall in similar cells.  A thread then takes
// one hit and a run of R phi0 rows (4 in 3D, 32 in 2D) and walks the d0
// slices upwards, keeping the hit's kappa bins of three slices (l - 1, l,
// l + 1) over rows j0 - 1 .. j0 + R in registers: every bin is computed once
// per thread, one new slice per step.  For a candidate row (l, jc) the hit's
// nine window bins b_p give the kappa bins it can reach, the union of
// [b_p - 1, b_p + 1]: the bitmap is read over [min b_p - 1, max b_p + 1], and
// each candidate found there is kept when some |b_p - kc| <= 1 -- so each
// (candidate, hit) pair is found once, by the thread that owns the
// candidate's row.  Each wavefront gathers its pairs (cell, hit) in LDS and
// reserves room in the output with one atomic per kAssocFlush pairs, looking
// up the candidate index of each cell as it writes them out.
#pragma clang fp contract(off)

#include <algorithm>

#include "assoc.h"
#include "vote_math.h"

namespace hough {
namespace {

constexpr int kAssocThreads = 256;
constexpr int kAssocWaves = kAssocThreads / 64;
constexpr int kAssocBuf = 512;      // pairs staged per wavefront
constexpr int kAssocFlush = kAssocBuf - 64;
constexpr int kSortBuckets = kAssocBuckets;

}  // namespace

// Bitmap dwords per (d0, phi0) row: bits 0 .. n_kappa + 1, plus one dword so
// that the pair of dwords holding any 32 consecutive bits never leaves the row.
int64_t assoc_row_words(int32_t n_kappa) {
    return (static_cast<int64_t>(n_kappa) + 2 + 31) / 32 + 1;
}

namespace {

struct AssocArgs {
    GridArgs g;
    const float4 *sorted;          // [n_hits] (x, y, x*x + y*y, hit index) in azimuth order
    int32_t n_hits;
    const int32_t *map;            // [cells] 1 + candidate index, 0: none
    const uint32_t *bits;          // [n_d0 * n_phi][row_words] bit kc + 1: a candidate at kc
    int32_t row_words;
    int32_t *pairs;                // [cap][2] (candidate, hit)
    int64_t cap;
    unsigned long long *n_pairs;
    int32_t approx;                // approximate bins with exact redos (phi0 table of bin centres, near_band > 0)
};

// Azimuth bucket of a hit (NaN and the origin go to bucket 0).
__device__ __forceinline__ int azimuth_bucket(float x, float y) {
    const float a = atan2f(y, x);                      // [-pi, pi]
    const float f = (a + 3.14159274f) * (kSortBuckets / 6.28318548f);
    const int b = f >= 0.0f ? static_cast<int>(f) : 0;  // NaN compares false
    return min(b, kSortBuckets - 1);
}

__global__ __launch_bounds__(kAssocThreads) void azimuth_hist_kernel(const float *x, const float *y, int32_t n,
                                                                      int32_t *hist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        atomicAdd(&hist[azimuth_bucket(x[i], y[i])], 1);
}

// Exclusive offsets of the buckets, in place (one workgroup of kSortBuckets threads).
__global__ __launch_bounds__(kSortBuckets) void azimuth_scan_kernel(int32_t *hist) {
    __shared__ int32_t s[kSortBuckets];
    const int t = threadIdx.x;
    const int v = hist[t];
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < kSortBuckets; off <<= 1) {
        const int w = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += w;
        __syncthreads();
    }
    hist[t] = s[t] - v;
}

__global__ __launch_bounds__(kAssocThreads) void azimuth_scatter_kernel(const float *x, const float *y, int32_t n,
                                                                         int32_t *offs, float4 *sorted) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float hx = x[i];
    const float hy = y[i];
    const int pos = atomicAdd(&offs[azimuth_bucket(hx, hy)], 1);
    sorted[pos] = make_float4(hx, hy, hx * hx + hy * hy, __int_as_float(i));
}

__global__ __launch_bounds__(kAssocThreads) void map_kernel(const Cand *cands, const int32_t *n_found, int32_t cap,
                                                            int32_t min_votes, int64_t cells, int32_t n_kappa,
                                                            int32_t row_words, int32_t *map, uint32_t *bits) {
    const int32_t n = min(*n_found, cap);
    for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const Cand cd = cands[c];
        if (cd.votes >= min_votes && cd.cell >= 0 && cd.cell < cells) {
            map[cd.cell] = c + 1;
            const int64_t row = cd.cell / n_kappa;
            const int b = cd.cell - static_cast<int32_t>(row * n_kappa) + 1;
            atomicOr(&bits[row * row_words + (b >> 5)], 1u << (b & 31));
        }
    }
}

// R phi0 rows per thread; D3: the grid has a d0 axis (slices l - 1 .. l + 1
// take part in a window), else one slice; STRAIGHT: the straight-line family;
// FWD: the forward-hemisphere option.
template <int R, bool D3, bool STRAIGHT, bool FWD>
__global__ __launch_bounds__(kAssocThreads) void assoc_kernel(AssocArgs a) {
    __shared__ int2 staged[kAssocWaves][kAssocBuf];
    const GridArgs &g = a.g;
    const int lane = threadIdx.x & 63;
    int2 *buf = staged[threadIdx.x >> 6];
    int fill = 0;                      // wave-uniform
    // move the staged pairs to the output: one reservation for all of them.
    // A staged pair holds the candidate's cell; its index comes from the
    // cell map here, one lookup per lane, so that the scan loop below never
    // waits on a load.  (A cell whose bitmap bit is set is a candidate's: the
    // map holds its index + 1 there.)
    auto flush = [&]() {
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (lane == 0)
            base = atomicAdd(a.n_pairs, static_cast<unsigned long long>(fill));
        base = __shfl(base, 0);
        for (int i = lane; i < fill; i += 64) {
            const int64_t slot = static_cast<int64_t>(base) + i;
            if (slot < a.cap) {
                const int2 p = buf[i];
                a.pairs[2 * slot] = a.map[p.x] - 1;
                a.pairs[2 * slot + 1] = p.y;
            }
        }
        __builtin_amdgcn_wave_barrier();
        fill = 0;
    };
    const int np = g.n_phi;
    const int nk = g.n_kappa;
    const int n_d0 = g.n_d0;
    const int j0 = blockIdx.x * R;
    const int i = blockIdx.y * kAssocThreads + threadIdx.x;
    const bool live = i < a.n_hits;
    const float4 rec = live ? a.sorted[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int h = __float_as_int(rec.w);
    const int64_t plane = static_cast<int64_t>(np) * nk;

    // The run's ring rows j0 - 1 .. j0 + R (cyclic) are the same for every
    // lane: u = y c - x s per row is computed once and serves every slice.
    const float kmin = g.kappa_min;
    const float kscale = g.kappa_scale;
    const float nkf = static_cast<float>(nk);
    float u[R + 2];
    bool votes[R + 2];                  // the hit exists (and, with the option, lies ahead)
#pragma unroll
    for (int k = 0; k < R + 2; ++k) {
        int row = j0 - 1 + k;
        row += row < 0 ? np : 0;
        row -= row >= np ? np : 0;
        const float c = g.cos_phi[row];
        const float sn = g.sin_phi[row];
        u[k] = rec.y * c - rec.x * sn;
        votes[k] = live;
        if constexpr (FWD) {
            const float ahead = rec.x * c + rec.y * sn;
            votes[k] = live && ahead > 0.0f;
        }
    }
    // The hit's kappa bins of slice ll over the ring rows: the vote of hough.h,
    // operation for operation (-1: no vote, or a slice outside the grid).
    auto exact_bin = [&](int k, bool ok, float d, float d2, float dd) {
        if constexpr (STRAIGHT) {
            const float kf = (u[k] - kmin) * kscale;
            return (ok && votes[k] && kf >= 0.0f && kf < nkf) ? static_cast<int>(kf) : -1;
        } else {
            const float num = 2.0f * (u[k] - d);
            const float den = (rec.z - d2 * u[k]) + dd;
            const float kappa = num / den;
            const float kf = (kappa - kmin) * kscale;
            return (ok && votes[k] && kf >= 0.0f && kf < nkf) ? static_cast<int>(kf) : -1;
        }
    };
    // The bins are kept biased: b + 1 for a vote in bin b, kNoBin for none.
    // Then kc is within one of b exactly when (b + 1) - kc, as unsigned, is at
    // most 2 -- kNoBin, far below zero, never is.
    constexpr int kNoBin = -(1 << 20);
    auto biased = [](int b) { return b >= 0 ? b + 1 : kNoBin; };
    // 2D: approximate bins with exact redos, as in the vote (vote_math.h):
    // kf1 = RN(u w + off) with the hit constant w = RN(y kappa_scale), y the
    // refined reciprocal of r2/2 (in the range of quot_den_ok), and the exact
    // bin only where kf1 lies within the band above an integer (the redo
    // divides with the operator).  The displaced grid keeps the exact form:
    // with u hoisted per row its quotient is not the larger part of a bin,
    // and the estimate measured slower there (4.03 against 3.85 ms on the
    // displaced event).
    const bool approx = !D3 && !STRAIGHT && a.approx != 0 && g.d0 == nullptr;
    const float band = g.near_band;
    const float kf_off = g.kf_off;
    const uint32_t lim_bits = __float_as_uint(nkf + 0.5f);
    const float half = 0.5f * rec.z;
    const bool fast2d = approx && quot_den_ok(half);
    const float w2d = fast2d ? quot_recip(half) * kscale : 0.0f;
    auto fill_slice = [&](int ll, int (&B)[R + 2]) {
        const bool ok = ll >= 0 && ll < n_d0;
        const float d = (ok && g.d0) ? g.d0[ll] : 0.0f;     // a one-slice grid may carry a d0 table
        const float d2 = 2.0f * d;
        const float dd = d * d;
        if (!approx) {
#pragma unroll
            for (int k = 0; k < R + 2; ++k)
                B[k] = biased(exact_bin(k, ok, d, d2, dd));
            return;
        }
        bool redo[R + 2];
        bool any = false;
#pragma unroll
        for (int k = 0; k < R + 2; ++k) {
            const float kf1 = kf_offset_2d(u[k], w2d, kf_off);
            const bool live = ok && votes[k];
            const float v = kf_clamp(live ? kf1 : __builtin_nanf(""), lim_bits);
            const int b = static_cast<int>(v);
            B[k] = b < nk ? b + 1 : kNoBin;
            redo[k] = live && (!fast2d || kf_in_band(v, band));
            any |= redo[k];
        }
        if (__ballot(any)) {
#pragma unroll
            for (int k = 0; k < R + 2; ++k)
                if (redo[k])
                    B[k] = biased(exact_bin(k, ok, d, d2, dd));
        }
    };
    int B0[R + 2], B1[R + 2], B2[R + 2];
#pragma unroll
    for (int k = 0; k < R + 2; ++k)
        B0[k] = kNoBin;
    fill_slice(0, B1);
    if constexpr (D3)
        fill_slice(1, B2);
    else
#pragma unroll
        for (int k = 0; k < R + 2; ++k)
            B2[k] = kNoBin;

    for (int l = 0; l < n_d0; ++l) {
        // column extremes over the three slices: the largest biased bin (kNoBin
        // never wins) and, as unsigned, the smallest valid one (kNoBin is
        // larger than any as unsigned)
        int cmax[R + 2];
        uint32_t cmin[R + 2];
#pragma unroll
        for (int k = 0; k < R + 2; ++k) {
            if constexpr (D3) {
                cmax[k] = max(max(B0[k], B1[k]), B2[k]);
                cmin[k] = min(min(static_cast<uint32_t>(B0[k]), static_cast<uint32_t>(B1[k])),
                              static_cast<uint32_t>(B2[k]));
            } else {
                cmax[k] = B1[k];
                cmin[k] = static_cast<uint32_t>(B1[k]);
            }
        }
        const uint32_t *brow0 = a.bits + static_cast<int64_t>(l) * np * a.row_words;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int jc = j0 + r;
            const int vmax = max(max(cmax[r], cmax[r + 1]), cmax[r + 2]);
            const uint32_t vmin_u = min(min(cmin[r], cmin[r + 1]), cmin[r + 2]);
            const bool any = jc < np && vmax >= 0;
            // candidates of row (l, jc) in [min b - 1, max b + 1] (b the
            // unbiased bins), 32 bins at a time
            const int k_lo = any ? max(static_cast<int>(vmin_u) - 2, 0) : 0;
            const int k_hi = any ? min(vmax, nk - 1) : -1;
            const uint32_t *brow = brow0 + static_cast<int64_t>(any ? jc : 0) * a.row_words;
            for (int base = k_lo; __ballot(base <= k_hi); base += 32) {
                uint32_t pend = 0u;
                if (base <= k_hi) {
                    // bits kc + 1 for kc = base .. base + 31
                    const int bit = base + 1;
                    const uint32_t *w = brow + (bit >> 5);
                    const uint64_t two = static_cast<uint64_t>(w[0]) | (static_cast<uint64_t>(w[1]) << 32);
                    pend = static_cast<uint32_t>(two >> (bit & 31));
                    const int width = k_hi - base + 1;
                    if (width < 32)
                        pend &= (1u << width) - 1u;
                }
                while (__ballot(pend != 0u)) {
                    bool emit = false;
                    int cell = 0;
                    if (pend != 0u) {
                        const int kc = base + (__ffs(pend) - 1);
                        pend &= pend - 1u;
                        // kept when a window bin is within one of kc
                        bool near = false;
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
                            near |= static_cast<uint32_t>(B1[r + t] - kc) <= 2u;
                            if constexpr (D3) {
                                near |= static_cast<uint32_t>(B0[r + t] - kc) <= 2u;
                                near |= static_cast<uint32_t>(B2[r + t] - kc) <= 2u;
                            }
                        }
                        emit = near;
                        cell = static_cast<int>(l * plane + static_cast<int64_t>(jc) * nk + kc);
                    }
                    const uint64_t m = __ballot(emit);
                    if (emit)
                        buf[fill + __popcll(m & ((1ull << lane) - 1ull))] = make_int2(cell, h);
                    fill += __popcll(m);
                    if (fill > kAssocFlush)
                        flush();
                }
            }
        }
        if constexpr (D3) {
#pragma unroll
            for (int k = 0; k < R + 2; ++k) {
                B0[k] = B1[k];
                B1[k] = B2[k];
            }
            if (l + 1 < n_d0)
                fill_slice(l + 2, B2);
        }
    }
    if (fill > 0)
        flush();
}

}  // namespace

hipError_t launch_associate(const GridArgs &g, const float *x, const float *y, int32_t n_hits, const Cand *cands,
                            const int32_t *n_found, int32_t cands_cap, int32_t min_votes, int32_t *map, uint32_t *bits,
                            float4 *sorted, int32_t *hist, int32_t *pairs, int64_t cap,
                            unsigned long long *n_pairs, bool approx, hipStream_t stream) {
    const int64_t row_words = assoc_row_words(g.n_kappa);
    hipError_t e = launch_zero(reinterpret_cast<uint32_t *>(map), g.cells, stream);
    if (e != hipSuccess)
        return e;
    e = launch_zero(bits, static_cast<int64_t>(g.n_d0) * g.n_phi * row_words, stream);
    if (e != hipSuccess)
        return e;
    e = launch_zero(reinterpret_cast<uint32_t *>(n_pairs), 2, stream);
    if (e != hipSuccess)
        return e;
    if (cands_cap > 0) {
        const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((cands_cap + kAssocThreads - 1) / kAssocThreads,
                                                                         4096));
        hipLaunchKernelGGL(map_kernel, dim3(blocks), dim3(kAssocThreads), 0, stream, cands, n_found, cands_cap,
                           min_votes, g.cells, g.n_kappa, static_cast<int32_t>(row_words), map, bits);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (n_hits == 0)
        return hipSuccess;
    // hits in azimuth order
    e = launch_zero(reinterpret_cast<uint32_t *>(hist), kSortBuckets, stream);
    if (e != hipSuccess)
        return e;
    const unsigned hb = static_cast<unsigned>((n_hits + kAssocThreads - 1) / kAssocThreads);
    hipLaunchKernelGGL(azimuth_hist_kernel, dim3(hb), dim3(kAssocThreads), 0, stream, x, y, n_hits, hist);
    hipLaunchKernelGGL(azimuth_scan_kernel, dim3(1), dim3(kSortBuckets), 0, stream, hist);
    hipLaunchKernelGGL(azimuth_scatter_kernel, dim3(hb), dim3(kAssocThreads), 0, stream, x, y, n_hits, hist, sorted);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    AssocArgs a{};
    a.g = g;
    a.sorted = sorted;
    a.n_hits = n_hits;
    a.map = map;
    a.bits = bits;
    a.row_words = static_cast<int32_t>(row_words);
    a.pairs = pairs;
    a.cap = cap;
    a.n_pairs = n_pairs;
    a.approx = approx && g.near_band > 0.0f ? 1 : 0;
    // rows per thread: measured best on the workload grids (2D 32, 3D 4)
    const bool d3 = g.n_d0 > 1;
    const int R = d3 ? 4 : 32;
    const dim3 grid(static_cast<unsigned>((g.n_phi + R - 1) / R), hb);
    auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, grid, dim3(kAssocThreads), 0, stream, a); };
    if (d3)
        g.forward ? go(assoc_kernel<4, true, false, true>) : go(assoc_kernel<4, true, false, false>);
    else if (g.straight)
        g.forward ? go(assoc_kernel<32, false, true, true>) : go(assoc_kernel<32, false, true, false>);
    else
        g.forward ? go(assoc_kernel<32, false, false, true>) : go(assoc_kernel<32, false, false, false>);
    return hipGetLastError();
}

}  // namespace hough
