// Hit association: the hits that make each track candidate (Section 3: a
// candidate is a local maximum of the votes cast by the hits compatible with
// it).  Hit h belongs to candidate C = (lc, jc, kc) when h votes into a cell
// of C's window (lc + dl, jc + dj, kc + dk), dl, dj, dk in {-1, 0, 1}: phi0
// modulo n_phi, d0 and kappa inside the grid -- the window of the peak rule.
//
// The vote is recomputed here in its plain binary32 form, operation for
// operation the definition in hough.h (this file is compiled with
// -ffp-contract=off; the division is the correctly rounded operator, the
// range test the compare form), with the grid's family and forward option.
//
// Layout: the context's cell map holds, per cell, 1 + the index of the
// candidate there (0: none).  One thread takes one (hit, d0 slice) and a run
// of kAssocRows phi0 rows; for every vote it looks up the candidates in the
// vote's window.  A pair is written once, by the first position of C's
// window (dl, then dj, in increasing order) at which the hit's bin is within
// one of kc: a thread that finds a match recomputes the hit's bins at the
// earlier positions of that window.  Pairs go out through one atomic
// reservation per wavefront.
#pragma clang fp contract(off)

#include "hough_impl.h"

namespace hough {
namespace {

constexpr int kAssocRows = 64;      // phi0 rows per thread
constexpr int kAssocThreads = 256;

struct AssocArgs {
    GridArgs g;
    const float *x, *y;
    int32_t n_hits;
    int32_t rows_chunks;           // ceil(n_phi / kAssocRows)
    const int32_t *map;            // [cells] 1 + candidate index, 0: none
    int32_t *pairs;                // [cap][2] (candidate, hit)
    int64_t cap;
    unsigned long long *n_pairs;
};

// The hit's kappa bin at (d0 slice l, phi0 row j), or -1 when it casts no vote there.
__device__ __forceinline__ int hit_bin(const GridArgs &g, float hx, float hy, float hr2, int l, int j) {
    const float c = g.cos_phi[j];
    const float s = g.sin_phi[j];
    if (g.forward) {
        const float ahead = hx * c + hy * s;
        if (!(ahead > 0.0f))
            return -1;
    }
    const float u = hy * c - hx * s;
    float kf;
    if (g.straight) {
        kf = (u - g.kappa_min) * g.kappa_scale;
    } else {
        const float d = g.d0 ? g.d0[l] : 0.0f;
        const float num = 2.0f * (u - d);
        const float den = hr2 - 2.0f * d * u + d * d;
        const float kappa = num / den;
        kf = (kappa - g.kappa_min) * g.kappa_scale;
    }
    return (kf >= 0.0f && kf < static_cast<float>(g.n_kappa)) ? static_cast<int>(kf) : -1;
}

__global__ __launch_bounds__(kAssocThreads) void map_kernel(const Cand *cands, const int32_t *n_found, int32_t cap,
                                                            int32_t min_votes, int64_t cells, int32_t *map) {
    const int32_t n = min(*n_found, cap);
    for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const Cand cd = cands[c];
        if (cd.votes >= min_votes && cd.cell >= 0 && cd.cell < cells)
            map[cd.cell] = c + 1;
    }
}

__global__ __launch_bounds__(kAssocThreads) void assoc_kernel(AssocArgs a) {
    const GridArgs &g = a.g;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per_hit = static_cast<int64_t>(g.n_d0) * a.rows_chunks;
    const int lane = threadIdx.x & 63;
    const bool live = t < per_hit * a.n_hits;
    const int h = live ? static_cast<int>(t / per_hit) : 0;
    const int rest = live ? static_cast<int>(t - static_cast<int64_t>(h) * per_hit) : 0;
    const int l = rest / a.rows_chunks;
    const int j0 = (rest - l * a.rows_chunks) * kAssocRows;
    const int j1 = live ? min(j0 + kAssocRows, g.n_phi) : j0;
    const float hx = live ? a.x[h] : 0.0f;
    const float hy = live ? a.y[h] : 0.0f;
    const float hr2 = hx * hx + hy * hy;
    const int nk = g.n_kappa;
    const int np = g.n_phi;
    const int64_t plane = static_cast<int64_t>(np) * nk;
    const int el_lo = g.n_d0 > 1 ? -1 : 0;
    const int el_hi = g.n_d0 > 1 ? 1 : 0;
    // every lane runs the same number of rows, so the wavefront stays together
    // for the reservations below
    for (int r = 0; r < kAssocRows; ++r) {
        const int j = j0 + r;
        const int k = j < j1 ? hit_bin(g, hx, hy, hr2, l, j) : -1;
        if (__ballot(k >= 0) == 0)
            continue;
        // candidates in the window of the vote (l, j, k): C = (l - el, j - ej, k - ek)
        for (int el = el_lo; el <= el_hi; ++el) {
            for (int ej = -1; ej <= 1; ++ej) {
                for (int ek = -1; ek <= 1; ++ek) {
                    const int lc = l - el;
                    int jc = j - ej;
                    jc += jc < 0 ? np : 0;
                    jc -= jc >= np ? np : 0;
                    const int kc = k - ek;
                    bool emit = false;
                    int cand = 0;
                    if (k >= 0 && lc >= 0 && lc < g.n_d0 && kc >= 0 && kc < nk) {
                        cand = a.map[lc * plane + static_cast<int64_t>(jc) * nk + kc] - 1;
                        if (cand >= 0) {
                            // the position (el, ej) of this vote in C's window; emit only when
                            // no earlier position of the window has the hit within one of kc
                            emit = true;
                            for (int dl = -1; dl <= el && emit; ++dl) {
                                const int ll = lc + dl;
                                if (ll < 0 || ll >= g.n_d0)
                                    continue;
                                for (int dj = -1; dj <= 1; ++dj) {
                                    if (dl == el && dj >= ej)
                                        break;
                                    int jj = jc + dj;
                                    jj += jj < 0 ? np : 0;
                                    jj -= jj >= np ? np : 0;
                                    const int kk = hit_bin(g, hx, hy, hr2, ll, jj);
                                    if (kk >= 0 && kk >= kc - 1 && kk <= kc + 1) {
                                        emit = false;
                                        break;
                                    }
                                }
                            }
                        }
                    }
                    const uint64_t m = __ballot(emit);
                    if (m) {
                        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
                        unsigned long long base = 0;
                        if (lane == leader)
                            base = atomicAdd(a.n_pairs, static_cast<unsigned long long>(__popcll(m)));
                        base = __shfl(base, leader);
                        if (emit) {
                            const int64_t slot = static_cast<int64_t>(base) + __popcll(m & ((1ull << lane) - 1ull));
                            if (slot < a.cap) {
                                a.pairs[2 * slot] = cand;
                                a.pairs[2 * slot + 1] = h;
                            }
                        }
                    }
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_associate(const GridArgs &g, const float *x, const float *y, int32_t n_hits, const Cand *cands,
                            const int32_t *n_found, int32_t cands_cap, int32_t min_votes, int32_t *map,
                            int32_t *pairs, int64_t cap, unsigned long long *n_pairs, hipStream_t stream) {
    hipError_t e = launch_zero(reinterpret_cast<uint32_t *>(map), g.cells, stream);
    if (e != hipSuccess)
        return e;
    e = launch_zero(reinterpret_cast<uint32_t *>(n_pairs), 2, stream);
    if (e != hipSuccess)
        return e;
    if (cands_cap > 0) {
        const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((cands_cap + kAssocThreads - 1) / kAssocThreads,
                                                                         4096));
        hipLaunchKernelGGL(map_kernel, dim3(blocks), dim3(kAssocThreads), 0, stream, cands, n_found, cands_cap,
                           min_votes, g.cells, map);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (n_hits == 0)
        return hipSuccess;
    AssocArgs a{};
    a.g = g;
    a.x = x;
    a.y = y;
    a.n_hits = n_hits;
    a.rows_chunks = (g.n_phi + kAssocRows - 1) / kAssocRows;
    a.map = map;
    a.pairs = pairs;
    a.cap = cap;
    a.n_pairs = n_pairs;
    const int64_t threads = static_cast<int64_t>(n_hits) * g.n_d0 * a.rows_chunks;
    const int64_t blocks = (threads + kAssocThreads - 1) / kAssocThreads;
    if (blocks > 0x7fffffffLL)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(assoc_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kAssocThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace hough
