// Peak search and candidate ordering for gfx950.
//
// Section 3: after voting, local maxima of the parameter space are the track
// candidates.  A block stages 16 phi0 rows of one d0 slice plus a one-row
// halo on each side (phi0 wraps) -- and the neighbouring d0 slices in 3D --
// in LDS, applies the threshold and the asymmetric 3x3(x3) local-maximum
// test of hough.h, and compacts the survivors in ascending cell order into
// its own staging list.  It also histograms the lowest sort digit and keeps
// the event's smallest and largest sort key.
//
// Ordering (votes descending, then cell ascending) is a stable LSD radix sort
// on key = 0x7fffffff - votes with 8-bit digits.  Staging lists are already
// in cell order, so a stable sort by key gives the required total order.
// Each pass is: per-chunk digit histogram, one scan per event turning the
// histograms into output offsets, and a scatter that ranks equal digits
// within a chunk in input order (wavefront ballots on the digit bits).  Only
// the digits in which an event's keys actually differ are sorted; the last
// pass writes straight into the caller's candidate array, clipped at its
// capacity.
#include "hough_impl.h"

namespace hough {
namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ int rank_below(uint64_t mask) {
    return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u)));
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = min(v, static_cast<uint32_t>(__shfl_xor(v, off, 64)));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = max(v, static_cast<uint32_t>(__shfl_xor(v, off, 64)));
    return v;
}

struct PeakArgs {
    GridArgs g;
    const uint32_t *acc;     // dwords, events back to back
    int32_t threshold;
    int32_t blocks_per_slice;
    SortWork w;
};

constexpr int kPeakThreads = 256;
constexpr int kHaloRows = kPeakRows + 2;

// LDS layout: [slice 0..2][row 0..kHaloRows-1][n_kappa] int32.
template <bool U16>
__global__ __launch_bounds__(kPeakThreads) void peak_kernel(PeakArgs a) {
    extern __shared__ int32_t tile[];
    __shared__ uint32_t hist[kDigits];
    __shared__ int32_t wave_cnt[kPeakThreads / 64];
    __shared__ uint32_t red_min[kPeakThreads / 64], red_max[kPeakThreads / 64];

    const GridArgs &g = a.g;
    const int tid = threadIdx.x;
    const int e = blockIdx.y;
    const int b = blockIdx.x;
    if (a.w.n_events_dev && e >= *a.w.n_events_dev)
        return;
    const int l = b / a.blocks_per_slice;
    const int j0 = (b - l * a.blocks_per_slice) * kPeakRows;
    const int rows_here = min(kPeakRows, g.n_phi - j0);
    const int nk = g.n_kappa;
    const int slice_cells = kHaloRows * nk;
    const bool has_lo = l > 0;
    const bool has_hi = l + 1 < g.n_d0;
    const bool three = g.n_d0 > 1;   // 2D grids stage only the middle slice

    for (int i = tid; i < kDigits; i += kPeakThreads)
        hist[i] = 0u;

    // Stage the rows j0-1 .. j0+rows_here of slices l-1, l, l+1.
    const uint32_t *acc_e = a.acc + static_cast<int64_t>(e) * g.acc_dwords;
    for (int sl = 0; sl < 3; ++sl) {
        const int ll = l + sl - 1;
        if (ll < 0 || ll >= g.n_d0)
            continue;
        for (int rr = 0; rr < rows_here + 2; ++rr) {
            int j = j0 + rr - 1;
            if (j < 0)
                j += g.n_phi;
            if (j >= g.n_phi)
                j -= g.n_phi;
            const uint32_t *src = acc_e + (static_cast<int64_t>(ll) * g.n_phi + j) * g.row_dwords;
            int32_t *dst = tile + (three ? sl : 0) * slice_cells + rr * nk;
            if constexpr (U16) {
                for (int w = tid; w < g.row_dwords; w += kPeakThreads) {
                    const uint32_t v = src[w];
                    dst[2 * w] = static_cast<int32_t>(v & 0xffffu);
                    dst[2 * w + 1] = static_cast<int32_t>(v >> 16);
                }
            } else {
                for (int w = tid; w < nk; w += kPeakThreads)
                    dst[w] = static_cast<int32_t>(src[w]);
            }
        }
    }
    __syncthreads();

    const int chunk = e * a.w.s0.n_chunks0 + b;
    Cand *out = a.w.s0.stage + static_cast<int64_t>(chunk) * a.w.s0.cap0;
    const int n_cells = rows_here * nk;
    uint32_t kmin = 0xffffffffu, kmax = 0u;
    int base = 0;
    const int wave = tid >> 6;
    for (int r0 = 0; r0 < n_cells; r0 += kPeakThreads) {
        const int idx = r0 + tid;
        bool keep = false;
        int32_t v = 0;
        int jr = 0, k = 0;
        if (idx < n_cells) {
            jr = idx / nk;
            k = idx - jr * nk;
            const int32_t *mid = tile + (three ? slice_cells : 0);
            v = mid[(jr + 1) * nk + k];
            keep = v >= a.threshold;
            if (keep) {
                // offsets in (d0, phi0, kappa) order; negative ones need v > w
                for (int od = -1; od <= 1 && keep; ++od) {
                    if ((od < 0 && !has_lo) || (od > 0 && !has_hi))
                        continue;
                    const int32_t *sl = tile + (three ? od + 1 : 0) * slice_cells;
                    for (int op = -1; op <= 1 && keep; ++op) {
                        const int32_t *row = sl + (jr + 1 + op) * nk;
                        for (int ok = -1; ok <= 1; ++ok) {
                            if (od == 0 && op == 0 && ok == 0)
                                continue;
                            const int kk = k + ok;
                            if (kk < 0 || kk >= nk)
                                continue;
                            const int32_t w = row[kk];
                            const bool neg = od != 0 ? od < 0 : (op != 0 ? op < 0 : ok < 0);
                            if (neg ? !(v > w) : !(v >= w)) {
                                keep = false;
                                break;
                            }
                        }
                    }
                }
            }
        }
        const uint64_t m = __ballot(keep);
        const int rank = rank_below(m);
        if (lane_id() == 0)
            wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int pre = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kPeakThreads / 64; ++w) {
            const int c = wave_cnt[w];
            pre += w < wave ? c : 0;
            total += c;
        }
        if (keep) {
            const int cell_local = (jr + j0) * nk + k;
            const int32_t cell = static_cast<int32_t>(static_cast<int64_t>(l) * g.n_phi * nk + cell_local);
            out[base + pre + rank] = Cand{v, cell};
            const uint32_t key = sort_key(v);
            atomicAdd(&hist[key & 0xffu], 1u);
            kmin = min(kmin, key);
            kmax = max(kmax, key);
        }
        base += total;
        __syncthreads();
    }

    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    if (lane_id() == 0) {
        red_min[wave] = kmin;
        red_max[wave] = kmax;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t mn = 0xffffffffu, mx = 0u;
        for (int w = 0; w < kPeakThreads / 64; ++w) {
            mn = min(mn, red_min[w]);
            mx = max(mx, red_max[w]);
        }
        a.w.s0.cnt0[chunk] = base;
        if (base > 0) {
            atomicMin(&a.w.state[e].key_min, mn);
            atomicMax(&a.w.state[e].key_max, mx);
        }
    }
    uint32_t *hrow = a.w.hist + (static_cast<int64_t>(e) * a.w.hist_chunks + b) * kDigits;
    for (int i = tid; i < kDigits; i += kPeakThreads)
        hrow[i] = hist[i];
}

// ---------------------------------------------------------------------------
// Radix sort passes
// ---------------------------------------------------------------------------

__device__ __forceinline__ int chunks_of(const SortWork &w, int pass, const EventState &st) {
    if (pass == 0)
        return w.s0.n_chunks0;
    return (st.n_found + kSortChunk - 1) / kSortChunk;
}

__device__ __forceinline__ const Cand *pass_source(const SortWork &w, int pass, int e, int c, int n_found,
                                                   int *count) {
    if (pass == 0) {
        const int chunk = e * w.s0.n_chunks0 + c;
        *count = w.s0.cnt0[chunk];
        return w.s0.stage + static_cast<int64_t>(chunk) * w.s0.cap0;
    }
    const Cand *buf = ((pass - 1) & 1) == 0 ? w.tmp0 : w.tmp1;
    const int begin = c * kSortChunk;
    *count = min(kSortChunk, n_found - begin);
    return buf + static_cast<int64_t>(e) * w.bound + begin;
}

// Digit histogram of one chunk of pass >= 1.
__global__ __launch_bounds__(kSortThreads) void hist_kernel(SortWork w, int pass) {
    __shared__ uint32_t hist[kDigits];
    const int e = blockIdx.y;
    const int c = blockIdx.x;
    if (w.n_events_dev && e >= *w.n_events_dev)
        return;
    const EventState st = w.state[e];
    if (pass >= st.passes || c >= chunks_of(w, pass, st))
        return;
    int count = 0;
    const Cand *src = pass_source(w, pass, e, c, st.n_found, &count);
    for (int i = threadIdx.x; i < kDigits; i += kSortThreads)
        hist[i] = 0u;
    __syncthreads();
    const int shift = 8 * pass;
    for (int i = threadIdx.x; i < count; i += kSortThreads)
        atomicAdd(&hist[(sort_key(src[i].votes) >> shift) & 0xffu], 1u);
    __syncthreads();
    uint32_t *hrow = w.hist + (static_cast<int64_t>(e) * w.hist_chunks + c) * kDigits;
    for (int i = threadIdx.x; i < kDigits; i += kSortThreads)
        hrow[i] = hist[i];
}

// Turn one event's [chunk][digit] histogram into exclusive output offsets
// (digit-major, chunk order within a digit).  Pass 0 also fixes n_found and
// the number of passes.
__global__ __launch_bounds__(kScanThreads) void scan_kernel(SortWork w, int pass) {
    constexpr int kGroups = kScanThreads / kDigits;
    __shared__ uint32_t part[kGroups][kDigits];
    __shared__ uint32_t base[kDigits];
    __shared__ uint32_t scan_tmp[kDigits];
    const int e = blockIdx.x;
    if (w.n_events_dev && e >= *w.n_events_dev)
        return;
    EventState st = w.state[e];
    if (pass > 0 && pass >= st.passes)
        return;
    int n_chunks;
    if (pass == 0) {
        n_chunks = w.s0.n_chunks0;
    } else {
        n_chunks = (st.n_found + kSortChunk - 1) / kSortChunk;
    }
    const int t = threadIdx.x;
    const int grp = t / kDigits;
    const int d = t % kDigits;
    const int per = (n_chunks + kGroups - 1) / kGroups;
    const int c_begin = min(n_chunks, grp * per);
    const int c_end = min(n_chunks, c_begin + per);
    uint32_t *h = w.hist + static_cast<int64_t>(e) * w.hist_chunks * kDigits;

    uint32_t sum = 0;
    for (int c = c_begin; c < c_end; ++c)
        sum += h[static_cast<int64_t>(c) * kDigits + d];
    part[grp][d] = sum;
    __syncthreads();
    if (grp == 0) {
        uint32_t tot = 0;
        for (int g2 = 0; g2 < kGroups; ++g2)
            tot += part[g2][d];
        scan_tmp[d] = tot;
    }
    __syncthreads();
    // inclusive Hillis-Steele scan over the 256 digit totals
    for (int off = 1; off < kDigits; off <<= 1) {
        uint32_t v = 0;
        if (grp == 0)
            v = scan_tmp[d] + (d >= off ? scan_tmp[d - off] : 0u);
        __syncthreads();
        if (grp == 0)
            scan_tmp[d] = v;
        __syncthreads();
    }
    if (grp == 0) {
        uint32_t tot = 0;
        for (int g2 = 0; g2 < kGroups; ++g2)
            tot += part[g2][d];
        base[d] = scan_tmp[d] - tot;
    }
    __syncthreads();
    if (pass == 0 && t == 0) {
        const int n_found = static_cast<int>(scan_tmp[kDigits - 1]);
        int passes = 1;
        if (n_found > 0) {
            const uint32_t diff = (st.key_min ^ st.key_max) & w.key_mask;
            if (diff)
                passes = (31 - __clz(diff)) / 8 + 1;
        }
        w.state[e].n_found = n_found;
        w.state[e].passes = passes;
        w.n_found[e] = n_found;
    }
    uint32_t run = base[d];
    for (int g2 = 0; g2 < grp; ++g2)
        run += part[g2][d];
    for (int c = c_begin; c < c_end; ++c) {
        const int64_t i = static_cast<int64_t>(c) * kDigits + d;
        const uint32_t v = h[i];
        h[i] = run;
        run += v;
    }
}

// Stable scatter of one chunk by the digit of this pass.
__global__ __launch_bounds__(kSortThreads) void scatter_kernel(SortWork w, int pass) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t run[kDigits];
    __shared__ uint32_t wcnt[kWaves][kDigits];
    const int e = blockIdx.y;
    const int c = blockIdx.x;
    if (w.n_events_dev && e >= *w.n_events_dev)
        return;
    const EventState st = w.state[e];
    if (pass >= st.passes || c >= chunks_of(w, pass, st))
        return;
    int count = 0;
    const Cand *src = pass_source(w, pass, e, c, st.n_found, &count);
    const bool last = pass == st.passes - 1;
    Cand *dst;
    int64_t limit;
    if (last) {
        if (w.desc) {
            dst = reinterpret_cast<Cand *>(w.out) + w.desc[e].cand_begin;
            limit = w.desc[e].cand_cap;
        } else {
            dst = reinterpret_cast<Cand *>(w.out);
            limit = w.cap;
        }
    } else {
        dst = ((pass & 1) == 0 ? w.tmp0 : w.tmp1) + static_cast<int64_t>(e) * w.bound;
        limit = w.bound;
    }
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const uint32_t *hrow = w.hist + (static_cast<int64_t>(e) * w.hist_chunks + c) * kDigits;
    for (int i = t; i < kDigits; i += kSortThreads)
        run[i] = hrow[i];
    const int shift = 8 * pass;
    for (int b0 = 0; b0 < count; b0 += kSortThreads) {
        for (int i = t; i < kWaves * kDigits; i += kSortThreads)
            (&wcnt[0][0])[i] = 0u;
        __syncthreads();
        const int i = b0 + t;
        const bool valid = i < count;
        Cand cd{0, 0};
        uint32_t digit = 0;
        if (valid) {
            cd = src[i];
            digit = (sort_key(cd.votes) >> shift) & 0xffu;
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (digit >> bit) & 1u;
            const uint64_t bb = __ballot(set);
            peers &= set ? bb : ~bb;
        }
        const int rank = rank_below(peers);
        if (valid && rank == 0)
            wcnt[wave][digit] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        if (valid) {
            uint32_t pre = run[digit];
            for (int w2 = 0; w2 < wave; ++w2)
                pre += wcnt[w2][digit];
            const int64_t pos = static_cast<int64_t>(pre) + rank;
            if (pos < limit)
                dst[pos] = cd;
        }
        __syncthreads();
        for (int dd = t; dd < kDigits; dd += kSortThreads) {
            uint32_t add = 0;
            for (int w2 = 0; w2 < kWaves; ++w2)
                add += wcnt[w2][dd];
            run[dd] += add;
        }
        __syncthreads();
    }
}

}  // namespace

int32_t peak_blocks_per_event(const GridArgs &g) {
    return g.n_d0 * ((g.n_phi + kPeakRows - 1) / kPeakRows);
}

int32_t peak_chunk_cap(const GridArgs &g) {
    // Survivors of one block form an independent set of the king's graph on
    // kPeakRows x n_kappa cells: at most ceil(rows/2) * ceil(n_kappa/2).
    return ((kPeakRows + 1) / 2) * ((g.n_kappa + 1) / 2);
}

hipError_t launch_peaks(const GridArgs &g, bool u16, const uint32_t *acc, int32_t n_events,
                        int32_t threshold, const SortWork &w, hipStream_t stream) {
    PeakArgs a{};
    a.g = g;
    a.acc = acc;
    a.threshold = threshold;
    a.blocks_per_slice = (g.n_phi + kPeakRows - 1) / kPeakRows;
    a.w = w;
    const size_t lds = static_cast<size_t>(g.n_d0 > 1 ? 3 : 1) * kHaloRows * g.n_kappa * sizeof(int32_t);
    const void *fn = u16 ? reinterpret_cast<const void *>(peak_kernel<true>)
                         : reinterpret_cast<const void *>(peak_kernel<false>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    dim3 grid(static_cast<unsigned>(peak_blocks_per_event(g)), static_cast<unsigned>(n_events));
    if (u16)
        hipLaunchKernelGGL(peak_kernel<true>, grid, dim3(kPeakThreads), lds, stream, a);
    else
        hipLaunchKernelGGL(peak_kernel<false>, grid, dim3(kPeakThreads), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_sort(const SortWork &w, int32_t n_events, hipStream_t stream) {
    const int max_passes = w.key_mask == 0xffffu ? 2 : kMaxPasses;
    const unsigned later_chunks = static_cast<unsigned>((w.bound + kSortChunk - 1) / kSortChunk);
    for (int pass = 0; pass < max_passes; ++pass) {
        if (pass > 0) {
            hipLaunchKernelGGL(hist_kernel, dim3(later_chunks, n_events), dim3(kSortThreads), 0, stream, w, pass);
        }
        hipLaunchKernelGGL(scan_kernel, dim3(n_events), dim3(kScanThreads), 0, stream, w, pass);
        const unsigned chunks = pass == 0 ? static_cast<unsigned>(w.s0.n_chunks0) : later_chunks;
        hipLaunchKernelGGL(scatter_kernel, dim3(chunks, n_events), dim3(kSortThreads), 0, stream, w, pass);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace hough
