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
// candidate there (0: none), and a bitmap of the cells that hold one: per
// (d0, phi0) row, bit kc + 1 of assoc_row_words(n_kappa) dwords (about 1 MB
// for the displaced grid, so it stays in L2).  One thread takes one (hit, d0
// slice l) and a run of kAssocRows phi0 rows, and owns the candidates of
// those cells.  Sliding along the rows it keeps the hit's bins at the nine
// window positions (slices l - 1 .. l + 1, rows jc - 1 .. jc + 1; three new
// bins per row in 3D, one in 2D); the candidates the hit reaches are the
// union of the positions' [b - 1, b + 1], read from two bitmap dwords per
// position, so each pair is found once without looking at other threads.
// Each wavefront gathers its pairs in an LDS buffer and reserves room in the
// output with one atomic per kAssocFlush pairs (a single counter taken per
// pair by every wavefront serialised the displaced event's 10^8 pairs).
#pragma clang fp contract(off)

#include "assoc.h"

namespace hough {
namespace {

constexpr int kAssocRows = 64;      // phi0 rows per thread
constexpr int kAssocThreads = 256;
constexpr int kAssocWaves = kAssocThreads / 64;
constexpr int kAssocBuf = 512;      // pairs staged per wavefront
constexpr int kAssocFlush = kAssocBuf - 64;

}  // namespace

// Bitmap dwords per (d0, phi0) row: bits 0 .. n_kappa + 1, plus one dword so
// that the pair of dwords holding bits k .. k + 2 never leaves the row.
int64_t assoc_row_words(int32_t n_kappa) {
    return (static_cast<int64_t>(n_kappa) + 2 + 31) / 32 + 1;
}

namespace {

struct AssocArgs {
    GridArgs g;
    const float *x, *y;
    int32_t n_hits;
    int32_t rows_chunks;           // ceil(n_phi / kAssocRows)
    const int32_t *map;            // [cells] 1 + candidate index, 0: none
    const uint32_t *bits;          // [n_d0 * n_phi][row_words] bit kc + 1: a candidate at kc
    int32_t row_words;
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

__global__ __launch_bounds__(kAssocThreads) void assoc_kernel(AssocArgs a) {
    __shared__ int2 staged[kAssocWaves][kAssocBuf];
    const GridArgs &g = a.g;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per_hit = static_cast<int64_t>(g.n_d0) * a.rows_chunks;
    const int lane = threadIdx.x & 63;
    int2 *buf = staged[threadIdx.x >> 6];
    int fill = 0;                      // wave-uniform
    // move the staged pairs to the output: one reservation for all of them
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
                a.pairs[2 * slot] = p.x;
                a.pairs[2 * slot + 1] = p.y;
            }
        }
        __builtin_amdgcn_wave_barrier();
        fill = 0;
    };
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
    // The thread owns the candidates C = (l, jc, kc) of its slice and rows.
    // The hit belongs to C when one of its bins b at the window positions
    // (l + dl, jc + dj) has |b - kc| <= 1, so the kc it reaches from row jc
    // form the union over the positions of [b - 1, b + 1]: each position adds
    // the candidates of its three cells that no earlier position covered, and
    // every pair comes out once.  bins[s][t]: slice l + s - 1, row jc + t - 1
    // (-1: no vote there, or a slice outside the grid), slid along the rows.
    int bins[3][3];
    auto bin_at = [&](int s, int row) -> int {
        const int ll = l + s - 1;
        if (!live || ll < 0 || ll >= g.n_d0)
            return -1;
        row += row < 0 ? np : 0;
        row -= row >= np ? np : 0;
        return hit_bin(g, hx, hy, hr2, ll, row);
    };
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        bins[s][0] = bin_at(s, j0 - 1);
        bins[s][1] = bin_at(s, j0);
    }
    const uint32_t *brow0 = a.bits + static_cast<int64_t>(l) * np * a.row_words;
    // every lane runs the same number of rows, so the wavefront stays together
    for (int r = 0; r < kAssocRows; ++r) {
        const int jc = j0 + r;
        const bool own = jc < j1;
#pragma unroll
        for (int s = 0; s < 3; ++s)
            bins[s][2] = own ? bin_at(s, jc + 1) : -1;
        const uint32_t *brow = brow0 + static_cast<int64_t>(own ? jc : 0) * a.row_words;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int kp = bins[p / 3][p % 3];
            uint32_t pend = 0u;
            if (own && kp >= 0) {
                // bits kc + 1 for kc = kp - 1 .. kp + 1 of the row (l, jc)
                const uint32_t *w = brow + (kp >> 5);
                const uint64_t two = static_cast<uint64_t>(w[0]) | (static_cast<uint64_t>(w[1]) << 32);
                pend = static_cast<uint32_t>(two >> (kp & 31)) & 7u;
                // minus the cells an earlier position already reached
                if (pend != 0u) {
#pragma unroll
                    for (int q = 0; q < p; ++q) {
                        const int kq = bins[q / 3][q % 3];
                        const int o = kq - kp;         // its cells are kp + o - 1 .. kp + o + 1
                        if (kq >= 0 && o >= -2 && o <= 2)
                            pend &= ~(o >= 0 ? (7u << o) : (7u >> -o));
                    }
                }
            }
            while (__ballot(pend != 0u)) {
                bool emit = false;
                int cand = 0;
                if (pend != 0u) {
                    const int kc = kp - 1 + (__ffs(pend) - 1);
                    pend &= pend - 1u;
                    cand = a.map[l * plane + static_cast<int64_t>(jc) * nk + kc] - 1;
                    emit = cand >= 0;
                }
                const uint64_t m = __ballot(emit);
                if (emit)
                    buf[fill + __popcll(m & ((1ull << lane) - 1ull))] = make_int2(cand, h);
                fill += __popcll(m);
                if (fill > kAssocFlush)
                    flush();
            }
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            bins[s][0] = bins[s][1];
            bins[s][1] = bins[s][2];
        }
    }
    if (fill > 0)
        flush();
}

}  // namespace

hipError_t launch_associate(const GridArgs &g, const float *x, const float *y, int32_t n_hits, const Cand *cands,
                            const int32_t *n_found, int32_t cands_cap, int32_t min_votes, int32_t *map, uint32_t *bits,
                            int32_t *pairs, int64_t cap, unsigned long long *n_pairs, hipStream_t stream) {
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
    AssocArgs a{};
    a.g = g;
    a.x = x;
    a.y = y;
    a.n_hits = n_hits;
    a.rows_chunks = (g.n_phi + kAssocRows - 1) / kAssocRows;
    a.map = map;
    a.bits = bits;
    a.row_words = static_cast<int32_t>(row_words);
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
