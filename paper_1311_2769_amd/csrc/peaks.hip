// Peak search and candidate ordering for gfx950.
//
// Section 3: after voting, local maxima of the parameter space are the track
// candidates.  A block stages kPeakRows phi0 rows of one d0 slice plus a
// one-row halo on each side (phi0 wraps) -- and the same rows of the
// neighbouring d0 slices in 3D -- in LDS, applies the threshold and the
// asymmetric 3x3(x3) local-maximum test of hough.h, and compacts the
// survivors in ascending cell order into its own staging list.
//
// Ordering (votes descending, then cell ascending) is a stable LSD radix sort
// on key = 0x7fffffff - votes with 8-bit digits.  Staging lists are already
// in cell order, so a stable sort by key gives the required total order.
// Each pass is: per-chunk digit histogram, one scan per event turning the
// histograms into output offsets, and a scatter that ranks equal digits
// within a chunk in input order (wavefront ballots on the digit bits).  In
// the first pass a chunk is a run of consecutive staging lists.  Only the
// digits in which an event's keys actually differ are sorted; the last pass
// writes straight into the caller's candidate array, clipped at its
// capacity.
#include "hough_impl.h"
#include "peak_tile.h"

namespace hough {
namespace {

struct PeakArgs {
    GridArgs g;
    const uint32_t *acc;     // dwords, events back to back
    int32_t threshold;
    int32_t blocks_per_slice;
    SortWork w;
};

constexpr int kPeakThreads = 256;
constexpr int kHaloRows = kPeakRows + 2;

// LDS layout: [slice 0..2][row 0..kHaloRows-1][n_kappa] int32 (2D: one slice).
template <bool U16>
__global__ __launch_bounds__(kPeakThreads) void peak_kernel(PeakArgs a) {
    extern __shared__ int32_t tile[];
    __shared__ CompactScratch<kPeakThreads> sc;

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
        sc.hist[i] = 0u;

    // Stage the rows j0-1 .. j0+rows_here of slices l-1, l, l+1.
    const uint32_t *acc_e = a.acc + static_cast<int64_t>(e) * g.acc_dwords;
    for (int sl = 0; sl < 3; ++sl) {
        const int ll = l + sl - 1;
        if (ll < 0 || ll >= g.n_d0)
            continue;
        int32_t *base = tile + (three ? sl : 0) * slice_cells;
        const int n_words = (rows_here + 2) * g.row_dwords;
        for (int i = tid; i < n_words; i += kPeakThreads) {
            const int rr = i / g.row_dwords;
            const int wd = i - rr * g.row_dwords;
            int j = j0 + rr - 1;
            if (j < 0)
                j += g.n_phi;
            if (j >= g.n_phi)
                j -= g.n_phi;
            const uint32_t v = acc_e[(static_cast<int64_t>(ll) * g.n_phi + j) * g.row_dwords + wd];
            int32_t *dst = base + rr * nk;
            if constexpr (U16) {
                dst[2 * wd] = static_cast<int32_t>(v & 0xffffu);
                dst[2 * wd + 1] = static_cast<int32_t>(v >> 16);
            } else {
                dst[wd] = static_cast<int32_t>(v);
            }
        }
    }
    __syncthreads();

    const int32_t *mid = tile + (three ? slice_cells : 0);
    const int32_t thr = a.threshold;
    const int64_t cell_base = static_cast<int64_t>(l) * g.n_phi * nk;
    auto test = [&](int idx, int32_t *v, int32_t *cell) {
        const int jr = idx / nk;
        const int k = idx - jr * nk;
        const int32_t *row = mid + (jr + 1) * nk;
        const int32_t val = row[k];
        if (val < thr || !is_peak_2d(row, nk, nk, k, val))
            return false;
        // d0 neighbours: the slice below is entirely "earlier" (v > w), the
        // slice above entirely "later" (v >= w).
        for (int od = -1; od <= 1; od += 2) {
            if ((od < 0 && !has_lo) || (od > 0 && !has_hi))
                continue;
            const int32_t *sl = tile + (od + 1) * slice_cells + jr * nk;   // row jr-1 of that slice
            for (int op = 0; op < 3; ++op) {
                const int32_t *rw = sl + op * nk;
                for (int ok = -1; ok <= 1; ++ok) {
                    const int kk = k + ok;
                    if (kk < 0 || kk >= nk)
                        continue;
                    const int32_t w = rw[kk];
                    if (od < 0 ? !(val > w) : !(val >= w))
                        return false;
                }
            }
        }
        *v = val;
        *cell = static_cast<int32_t>(cell_base + static_cast<int64_t>(j0 + jr) * nk + k);
        return true;
    };
    Cand *out = a.w.s0.stage + (static_cast<int64_t>(e) * a.w.s0.n_blocks0 + b) * a.w.s0.cap0;
    uint32_t kmin, kmax;
    const int count = compact_ordered<kPeakThreads>(rows_here * nk, test, out, sc, &kmin, &kmax);
    publish_block<kPeakThreads>(a.w, e, b, count, sc, kmin, kmax);
}

// ---------------------------------------------------------------------------
// Radix sort passes
// ---------------------------------------------------------------------------

__device__ __forceinline__ int chunks_of(const SortWork &w, int pass, const EventState &st) {
    if (pass == 0)
        return (w.s0.n_blocks0 + w.s0.cb - 1) / w.s0.cb;
    return (st.n_found + kSortChunk - 1) / kSortChunk;
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
    const Cand *buf = ((pass - 1) & 1) == 0 ? w.tmp0 : w.tmp1;
    const int begin = c * kSortChunk;
    const int count = min(kSortChunk, st.n_found - begin);
    const Cand *src = buf + static_cast<int64_t>(e) * w.bound + begin;
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
    const int n_chunks = chunks_of(w, pass, st);
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

    // The chunk's input: pass 0 reads cb consecutive staging lists, later
    // passes one contiguous range of the previous pass's output.
    int n_lists = 1;
    int b_first = 0;
    if (pass == 0) {
        b_first = c * w.s0.cb;
        n_lists = min(w.s0.cb, w.s0.n_blocks0 - b_first);
    }
    for (int li = 0; li < n_lists; ++li) {
        const Cand *src;
        int count;
        if (pass == 0) {
            const int64_t blk = static_cast<int64_t>(e) * w.s0.n_blocks0 + b_first + li;
            src = w.s0.stage + blk * w.s0.cap0;
            count = w.s0.cnt0[blk];
        } else {
            const Cand *buf = ((pass - 1) & 1) == 0 ? w.tmp0 : w.tmp1;
            const int begin = c * kSortChunk;
            count = min(kSortChunk, st.n_found - begin);
            src = buf + static_cast<int64_t>(e) * w.bound + begin;
        }
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
}

}  // namespace

int32_t peak_blocks_per_event(const GridArgs &g) {
    return g.n_d0 * ((g.n_phi + kPeakRows - 1) / kPeakRows);
}

int32_t peak_block_cap(const GridArgs &g) {
    // Survivors of one block form an independent set of the king's graph on
    // kPeakRows x n_kappa cells: at most ceil(rows/2) * ceil(n_kappa/2).
    return ((kPeakRows + 1) / 2) * ((g.n_kappa + 1) / 2);
}

int32_t peak_blocks_per_chunk(const GridArgs &g) {
    // At most 256 first-pass chunks per event keeps the offset scan short.
    const int32_t blocks = peak_blocks_per_event(g);
    return (blocks + 255) / 256;
}

hipError_t launch_peaks(const GridArgs &g, bool u16, const uint32_t *acc, int32_t n_events,
                        int32_t threshold, const SortWork &w, hipStream_t stream) {
    PeakArgs a{};
    a.g = g;
    a.acc = acc;
    a.threshold = threshold;
    a.blocks_per_slice = (g.n_phi + kPeakRows - 1) / kPeakRows;
    a.w = w;
    if (w.s0.cb > 1) {
        // blocks add into shared first-pass histogram rows
        hipError_t e = launch_zero(w.hist, static_cast<int64_t>(n_events) * w.hist_chunks * kDigits, stream);
        if (e != hipSuccess)
            return e;
    }
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
    const unsigned first_chunks = static_cast<unsigned>((w.s0.n_blocks0 + w.s0.cb - 1) / w.s0.cb);
    for (int pass = 0; pass < max_passes; ++pass) {
        if (pass > 0)
            hipLaunchKernelGGL(hist_kernel, dim3(later_chunks, n_events), dim3(kSortThreads), 0, stream, w, pass);
        hipLaunchKernelGGL(scan_kernel, dim3(n_events), dim3(kScanThreads), 0, stream, w, pass);
        const unsigned chunks = pass == 0 ? first_chunks : later_chunks;
        hipLaunchKernelGGL(scatter_kernel, dim3(chunks, n_events), dim3(kSortThreads), 0, stream, w, pass);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace hough
