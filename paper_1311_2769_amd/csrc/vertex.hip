// Displaced vertices: the second Hough transform (Section 5).
//
// The first transform's candidates are tracks; a vertex V is the sinusoid
// d0 = V_y cos(phi0) - V_x sin(phi0) of the (phi0, d0) plane, so every track
// candidate with at least track_threshold votes is read as the straight line
// of vertices V with V_y c - V_x s = d0 (c, s, d0 the bin centres of its
// cell) and votes into a binned (x, y) vertex grid: once per column when
// |c| >= |s| (the line's y at the column centre), else once per row (its x at
// the row centre).  Arithmetic is the fp32 definition of hough.h, operation
// for operation (this file is compiled with -ffp-contract=off):
//     column ix:  y = (d0 + x_centre[ix] * s) / c,  fy = (y - y_min) * y_scale
//     row iy:     x = (y_centre[iy] * c - d0) / s,  fx = (x - x_min) * x_scale
// with a vote when the fractional bin lies in [0, n).  Vertex candidates are
// the cells that reach vertex_threshold and pass the asymmetric 3x3 local-
// maximum rule with neither axis periodic, sorted by votes descending then
// cell (ix * n_y + iy) ascending.
//
// One workgroup per event holds the event's whole vertex accumulator in LDS
// (at most kVtxMaxCells cells).  It reads the candidates in coalesced rounds
// and lists the ones that vote; wavefronts then take lines and lanes the
// columns or rows of a line, each vote an LDS atomic.  A list sorted by
// votes (as the first transform writes it) ends its scan at the first
// candidate below the track threshold.  The peak test runs over LDS;
// survivors are packed as 64-bit keys (0x7fffffff - votes, cell),
// bitonic-sorted in LDS and written out.  (Spreading one event over many
// workgroups with atomics into memory measured 4x slower.)
#pragma clang fp contract(off)

#include <climits>

#include "hough_impl.h"
#include "peak_tile.h"

namespace hough {
namespace {

constexpr int kVtxThreads = 1024;
constexpr int kVtxWaves = kVtxThreads / 64;
constexpr int kVtxPer = 4;                          // candidates per thread per round
constexpr int kVtxScan = kVtxPer * kVtxThreads;     // candidates per round
constexpr int kVtxRegCentres = 4;                   // centres per lane kept in registers (axes <= 256 bins)

struct VertexArgs {
    GridArgs g;                   // the track grid of the candidates
    const Cand *cands;            // [dev] first-transform candidates, events back to back
    const int64_t *cand_off;      // [dev][n_events + 1] list slices
    const int32_t *n_found;       // [dev][n_events] candidates found (may exceed the slice)
    int32_t track_threshold;
    int32_t vertex_threshold;
    int32_t sorted;               // lists sorted by votes descending: stop at the first below threshold
    int32_t n_x, n_y;
    float x_min, x_scale, y_min, y_scale;
    const float *x_centre;        // [dev][n_x]
    const float *y_centre;        // [dev][n_y]
    int32_t sort_size;            // power of two >= the survivor bound
    Cand *vout;                   // [dev] vertex candidates
    const int64_t *vout_off;      // [dev][n_events + 1]
    int32_t *n_vertices;          // [dev][n_events]
    int32_t *vacc;                // [dev][n_events][n_x * n_y] or nullptr
};

__global__ __launch_bounds__(kVtxThreads) void vertex_kernel(VertexArgs a) {
    extern __shared__ uint64_t vtx_lds[];
    __shared__ int32_t n_peaks;
    __shared__ int32_t n_lines;
    __shared__ float3 lines[kVtxScan];    // (d0, cos phi0, sin phi0) of the round's voting candidates
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int n_x = a.n_x;
    const int n_y = a.n_y;
    const int cells = n_x * n_y;
    // LDS columns are n_y + 1 dwords apart: the 64 lanes of a shallow line add
    // into 64 consecutive columns, which would otherwise share one bank
    const int ys = n_y + 1;
    uint64_t *keys = vtx_lds;                                              // [sort_size]
    int32_t *acc = reinterpret_cast<int32_t *>(vtx_lds + a.sort_size);     // [n_x][ys]

    for (int i = tid; i < n_x * ys; i += kVtxThreads)
        acc[i] = 0;
    if (tid == 0) {
        n_peaks = 0;
        n_lines = 0;
    }

    // Votes, in rounds of kVtxScan candidates: the workgroup reads a round
    // (coalesced; the next round is loaded while this one votes), lists the
    // lines that vote, then a wavefront per line casts it with its lanes
    // across the columns or rows.  Integer counts do not depend on the order
    // of the votes.
    const GridArgs &g = a.g;
    const int64_t begin = a.cand_off[e];
    const int64_t room = a.cand_off[e + 1] - begin;
    const int64_t found = a.n_found[e];
    const int64_t n = found < room ? found : room;
    const int64_t track_cells = g.cells;
    const int plane = g.n_phi * g.n_kappa;
    const float nxf = static_cast<float>(n_x);
    const float nyf = static_cast<float>(n_y);
    // the column and row centres of this lane (the same for every line)
    float xcr[kVtxRegCentres], ycr[kVtxRegCentres];
#pragma unroll
    for (int k = 0; k < kVtxRegCentres; ++k) {
        xcr[k] = lane + 64 * k < n_x ? a.x_centre[lane + 64 * k] : 0.0f;
        ycr[k] = lane + 64 * k < n_y ? a.y_centre[lane + 64 * k] : 0.0f;
    }
    Cand pf[kVtxPer];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < kVtxPer; ++q) {
            const int64_t i = r0 + q * kVtxThreads + tid;
            pf[q] = i < n ? a.cands[begin + i] : Cand{INT_MIN, -1};
        }
    };
    fetch(0);
    __syncthreads();
    for (int64_t r0 = 0; r0 < n; r0 += kVtxScan) {
        bool below = false;
#pragma unroll
        for (int q = 0; q < kVtxPer; ++q) {
            const Cand cd = pf[q];
            const bool live = r0 + q * kVtxThreads + tid < n;
            below = below || (live && cd.votes < a.track_threshold);
            // (cells outside the grid are never produced by the first transform);
            // one slot reservation per wavefront, and the line's constants are
            // loaded here, by every lister at once
            const bool vote = cd.votes >= a.track_threshold && cd.cell >= 0 && cd.cell < track_cells;
            const uint64_t mask = __ballot(vote);
            int base = 0;
            if (lane == 0 && mask)
                base = atomicAdd(&n_lines, __popcll(mask));
            base = __builtin_amdgcn_readfirstlane(base);
            if (vote) {
                const int l = cd.cell / plane;
                const int j = (cd.cell / g.n_kappa) % g.n_phi;
                lines[base + rank_below(mask)] = make_float3(g.d0 ? g.d0[l] : 0.0f, g.cos_phi[j], g.sin_phi[j]);
            }
        }
        // a sorted list has no voting candidate after its first one below threshold
        const bool last = __syncthreads_or(a.sorted && below) != 0;
        if (!last && r0 + kVtxScan < n)
            fetch(r0 + kVtxScan);
        const int m = n_lines;
        for (int li = wave; li < m; li += kVtxWaves) {
            const float3 ln = lines[li];
            const float dt = ln.x;
            const float c = ln.y;
            const float s = ln.z;
            auto col = [&](int ix, float xc) {
                const float t = xc * s;
                const float num = dt + t;
                const float yv = num / c;
                const float fy = (yv - a.y_min) * a.y_scale;
                if (fy >= 0.0f && fy < nyf)
                    atomicAdd(&acc[ix * ys + static_cast<int>(fy)], 1);
            };
            auto row = [&](int iy, float yc) {
                const float t = yc * c;
                const float num = t - dt;
                const float xv = num / s;
                const float fx = (xv - a.x_min) * a.x_scale;
                if (fx >= 0.0f && fx < nxf)
                    atomicAdd(&acc[static_cast<int>(fx) * ys + iy], 1);
            };
            if (fabsf(c) >= fabsf(s)) {
#pragma unroll
                for (int k = 0; k < kVtxRegCentres; ++k) {
                    if (lane + 64 * k < n_x)
                        col(lane + 64 * k, xcr[k]);
                }
                for (int ix = lane + 64 * kVtxRegCentres; ix < n_x; ix += 64)
                    col(ix, a.x_centre[ix]);
            } else {
#pragma unroll
                for (int k = 0; k < kVtxRegCentres; ++k) {
                    if (lane + 64 * k < n_y)
                        row(lane + 64 * k, ycr[k]);
                }
                for (int iy = lane + 64 * kVtxRegCentres; iy < n_y; iy += 64)
                    row(iy, a.y_centre[iy]);
            }
        }
        __syncthreads();
        if (tid == 0)
            n_lines = 0;
        __syncthreads();
        if (last)
            break;
    }

    if (a.vacc) {
        int32_t *dst = a.vacc + static_cast<int64_t>(e) * cells;
        for (int i = tid; i < cells; i += kVtxThreads) {
            const int ix = i / n_y;
            dst[i] = acc[i + ix];
        }
    }

    // peaks: neighbours outside the grid are ignored; earlier offsets (dx, dy)
    // must be exceeded, later ones reached
    for (int cell = tid; cell < cells; cell += kVtxThreads) {
        const int ix = cell / n_y;
        const int iy = cell - ix * n_y;
        const int32_t v = acc[ix * ys + iy];
        if (v < a.vertex_threshold)
            continue;
        bool keep = true;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                if (dx == 0 && dy == 0)
                    continue;
                const int xx = ix + dx;
                const int yy = iy + dy;
                if (xx < 0 || xx >= n_x || yy < 0 || yy >= n_y)
                    continue;
                const int32_t w = acc[xx * ys + yy];
                const bool earlier = dx < 0 || (dx == 0 && dy < 0);
                keep = keep && (earlier ? v > w : v >= w);
            }
        }
        // one slot reservation per wavefront, by its lowest surviving lane
        const uint64_t pm = __ballot(keep);
        if (keep) {
            const int leader = __ffsll(static_cast<unsigned long long>(pm)) - 1;
            int base = 0;
            if (lane == leader)
                base = atomicAdd(&n_peaks, __popcll(pm));
            base = __shfl(base, leader);
            // survivors are at most sort_size (host-checked independence bound)
            const int slot = base + __popcll(pm & ((1ull << lane) - 1ull));
            if (slot < a.sort_size)
                keys[slot] = (static_cast<uint64_t>(0x7fffffffu - static_cast<uint32_t>(v)) << 32) |
                             static_cast<uint32_t>(cell);
        }
    }
    __syncthreads();
    const int m = min(n_peaks, a.sort_size);
    int P = 1;
    while (P < m)
        P <<= 1;
    for (int i = m + tid; i < P; i += kVtxThreads)
        keys[i] = ~0ull;
    __syncthreads();
    // bitonic sort of keys[0, P) ascending
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = tid; i < P; i += kVtxThreads) {
                const int p = i ^ jj;
                if (p > i) {
                    const uint64_t ki = keys[i];
                    const uint64_t kp = keys[p];
                    const bool up = (i & k) == 0;
                    if (up ? ki > kp : ki < kp) {
                        keys[i] = kp;
                        keys[p] = ki;
                    }
                }
            }
            __syncthreads();
        }
    }

    const int64_t vbegin = a.vout_off[e];
    const int64_t vroom = a.vout_off[e + 1] - vbegin;
    const int64_t n_out = m < vroom ? m : vroom;
    for (int64_t i = tid; i < n_out; i += kVtxThreads) {
        const uint64_t key = keys[i];
        a.vout[vbegin + i] = Cand{static_cast<int32_t>(0x7fffffffu - static_cast<uint32_t>(key >> 32)),
                                  static_cast<int32_t>(key & 0xffffffffu)};
    }
    if (tid == 0)
        a.n_vertices[e] = n_peaks;
}

}  // namespace

int32_t vertex_sort_size(int32_t n_x, int32_t n_y) {
    // survivors form an independent set of the king's graph on the grid
    const int64_t bound = static_cast<int64_t>((n_x + 1) / 2) * ((n_y + 1) / 2);
    int32_t p = 1;
    while (p < bound)
        p <<= 1;
    return p;
}

bool vertex_grid_supported(int32_t n_x, int32_t n_y) {
    if (n_x < 1 || n_y < 1 || static_cast<int64_t>(n_x) * n_y > kVtxMaxCells || vertex_sort_size(n_x, n_y) > kVtxMaxPeaks)
        return false;
    const size_t lds = static_cast<size_t>(vertex_sort_size(n_x, n_y)) * sizeof(uint64_t) +
                       static_cast<size_t>(n_x) * (n_y + 1) * sizeof(int32_t) + kVtxScan * sizeof(float3) + 64;
    return lds <= 160u * 1024u;
}

hipError_t launch_vertices(const GridArgs &g, const hough_vertex_grid &vg, int32_t n_events, const Cand *cands,
                           const int64_t *cand_off, const int32_t *n_found, int32_t track_threshold,
                           int32_t vertex_threshold, int32_t sorted, Cand *vout, const int64_t *vout_off,
                           int32_t *n_vertices, int32_t *vacc, hipStream_t stream) {
    VertexArgs a{};
    a.g = g;
    a.cands = cands;
    a.cand_off = cand_off;
    a.n_found = n_found;
    a.track_threshold = track_threshold;
    a.vertex_threshold = vertex_threshold;
    a.sorted = sorted ? 1 : 0;
    a.n_x = vg.n_x;
    a.n_y = vg.n_y;
    a.x_min = vg.x_min;
    a.x_scale = vg.x_scale;
    a.y_min = vg.y_min;
    a.y_scale = vg.y_scale;
    a.x_centre = vg.x_centre;
    a.y_centre = vg.y_centre;
    a.sort_size = vertex_sort_size(vg.n_x, vg.n_y);
    a.vout = vout;
    a.vout_off = vout_off;
    a.n_vertices = n_vertices;
    a.vacc = vacc;
    const size_t lds = static_cast<size_t>(a.sort_size) * sizeof(uint64_t) +
                       static_cast<size_t>(vg.n_x) * (vg.n_y + 1) * sizeof(int32_t);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(vertex_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(vertex_kernel, dim3(static_cast<unsigned>(n_events)), dim3(kVtxThreads), lds, stream, a);
    return hipGetLastError();
}

}  // namespace hough
