// Peak search and candidate ordering for gfx950.
//
// Section 3: after voting, local maxima of the parameter space are the track
// candidates.  A block owns a band of kPeakRows phi0 rows and walks
// kPeakSlices consecutive d0 slices of it, keeping three slices (d0 l-1, l,
// l+1) of the band plus a one-row halo on each side (phi0 wraps) in an LDS
// ring, so each slice is read from memory about (kPeakSlices + 2) /
// kPeakSlices times.  uint16 cells are unpacked to int32; every staged row is
// padded with one INT_MIN column on each side, which stands for the kappa
// neighbours outside the grid (never larger than a cell).  For slice l the
// asymmetric 3x3(x3) test of hough.h is branch-free: the cell must exceed the
// maximum of its lexicographically earlier neighbours -- the whole slice
// below, the row above, the cell to its left -- and reach the maximum of the
// later ones.  Survivors of each (slice, band) are compacted in ascending
// cell order into that pair's staging list.
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
#include <climits>

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
constexpr int kPeakWaves = kPeakThreads / 64;
constexpr int kHaloRows = kPeakRows + 2;
constexpr int kPeakSlices = 8;
constexpr int kPrefetch = 8;                              // dwords per thread per load round
constexpr int kMaxSegs = 64;                              // (row, kappa chunk) pairs per band

__device__ __forceinline__ int32_t max3i(int32_t a, int32_t b, int32_t c) { return max(max(a, b), c); }

struct PeakScratch {
    uint32_t hist[kDigits];
    uint64_t seg_mask[kMaxSegs][kPeakWaves];   // survivor lanes per (row, kappa chunk) and wavefront
    uint32_t red_min[kPeakWaves];
    uint32_t red_max[kPeakWaves];
};

// LDS: a ring of 4 slices (2D: 1) x kHaloRows rows x (n_kappa + 2) int32,
// then two dwords per thread that take the stores of positions past the band.
// The slice after next is loaded into registers while the current slice is
// tested and stored into the ring afterwards, so its memory latency overlaps
// the test.
template <bool U16>
__global__ __launch_bounds__(kPeakThreads) void peak_kernel(PeakArgs a) {
    extern __shared__ int32_t ring[];
    __shared__ PeakScratch sc;

    const GridArgs &g = a.g;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int e = blockIdx.y;
    if (a.w.n_events_dev && e >= *a.w.n_events_dev)
        return;
    const int bps = a.blocks_per_slice;
    const int rb = blockIdx.x % bps;
    const int l0 = (blockIdx.x / bps) * kPeakSlices;
    const int l1 = min(g.n_d0, l0 + kPeakSlices);
    const int j0 = rb * kPeakRows;
    const int rows_here = min(kPeakRows, g.n_phi - j0);
    const int nk = g.n_kappa;
    const int W = nk + 2;
    const int plane = kHaloRows * W;
    const bool three = g.n_d0 > 1;
    const int rd = g.row_dwords;
    const int n_words = (rows_here + 2) * rd;             // staged dwords of one slice
    const uint32_t *acc_e = a.acc + static_cast<int64_t>(e) * g.acc_dwords;
    auto slot = [&](int ll) { return ring + (three ? (ll & 3) : 0) * plane; };

    // Staged dword i = tid + kPeakThreads*m of a band is (row rr, dword wd)
    // with i = rr*rd + wd.  For the first load round (all of it when the band
    // fits one round) each thread's global and LDS offsets are the same for
    // every slice, so they are computed once.
    const int dr = kPeakThreads / rd;
    const int dw = kPeakThreads - dr * rd;
    const int rr_first = tid / rd;
    const int wd_first = tid - rr_first * rd;
    auto advance = [&](int &rr, int &wd) {
        wd += dw;
        rr += dr;
        if (wd >= rd) {
            wd -= rd;
            ++rr;
        }
    };
    // Positions past the band load dword 0 of the slice and store into this
    // thread's own two dwords after the ring, so the rounds need no branches.
    int32_t goff[kPrefetch];   // dword offset inside a slice
    int32_t loff[kPrefetch];   // LDS offset of the first staged cell, from the ring base
    const int slot_words = (three ? 4 : 1) * plane;
    {
        int rr = rr_first, wd = wd_first;
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
            int j = j0 + rr - 1;
            j += j < 0 ? g.n_phi : 0;
            j -= j >= g.n_phi ? g.n_phi : 0;
            const bool in = rr < rows_here + 2;
            goff[q] = in ? j * rd + wd : 0;
            loff[q] = in ? rr * W + 1 + (U16 ? 2 * wd : wd) : -1;
            advance(rr, wd);
        }
    }
    int32_t *const dummy = ring + slot_words + 2 * tid;
    uint32_t pv[kPrefetch];
    auto issue_first = [&](int ll) {
        const uint32_t *src = acc_e + static_cast<int64_t>(ll) * g.n_phi * rd;
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q)
            pv[q] = src[goff[q]];
    };
    auto commit_first = [&](int ll) {
        int32_t *p = slot(ll);
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
            int32_t *d = loff[q] >= 0 ? p + loff[q] : dummy;
            if constexpr (U16) {
                d[0] = static_cast<int32_t>(pv[q] & 0xffffu);
                d[1] = static_cast<int32_t>(pv[q] >> 16);
            } else {
                d[0] = static_cast<int32_t>(pv[q]);
            }
        }
    };
    auto pad = [&](int ll) {
        int32_t *p = slot(ll);
        for (int rr = tid; rr < kHaloRows; rr += kPeakThreads) {
            p[rr * W] = INT_MIN;
            p[rr * W + nk + 1] = INT_MIN;
        }
    };
    auto load = [&](int ll) {
        issue_first(ll);
        commit_first(ll);
        // rounds after the first
        int rr = rr_first, wd = wd_first;
        for (int q = 0; q < kPrefetch; ++q)
            advance(rr, wd);
        for (int c0 = kPrefetch * kPeakThreads; c0 < n_words; c0 += kPrefetch * kPeakThreads) {
            const uint32_t *src = acc_e + static_cast<int64_t>(ll) * g.n_phi * rd;
            int32_t *p = slot(ll);
            for (int q = 0; q < kPrefetch; ++q) {
                if (rr < rows_here + 2) {
                    int j = j0 + rr - 1;
                    j += j < 0 ? g.n_phi : 0;
                    j -= j >= g.n_phi ? g.n_phi : 0;
                    const uint32_t v = src[static_cast<int64_t>(j) * rd + wd];
                    int32_t *dst = p + rr * W + 1;
                    if constexpr (U16) {
                        dst[2 * wd] = static_cast<int32_t>(v & 0xffffu);
                        dst[2 * wd + 1] = static_cast<int32_t>(v >> 16);
                    } else {
                        dst[wd] = static_cast<int32_t>(v);
                    }
                }
                advance(rr, wd);
            }
        }
        pad(ll);
    };
    // The slice after next can stay in registers across the test when it fits one round.
    const bool overlap = three && n_words <= kPrefetch * kPeakThreads;

    if (three && l0 > 0)
        load(l0 - 1);
    load(l0);
    if (three && l0 + 1 < g.n_d0)
        load(l0 + 1);
    const int32_t thr = a.threshold;
    // rows_here * ceil(nk / kPeakThreads) segments <= kMaxSegs (checked on the host)
    for (int l = l0; l < l1; ++l) {
        const bool next2 = three && l + 2 < g.n_d0 && l + 2 <= l1;   // needed by this block's last step
        if (next2 && overlap)
            issue_first(l + 2);
        for (int i = tid; i < kDigits; i += kPeakThreads)
            sc.hist[i] = 0u;
        lds_barrier();
        const bool has_lo = three && l > 0;
        const bool has_hi = three && l + 1 < g.n_d0;
        const int32_t *mid = slot(l);
        const int32_t *lo = slot(has_lo ? l - 1 : l);
        const int32_t *hi = slot(has_hi ? l + 1 : l);

        // Test of cell (row jr of the band, kappa k); cells in ascending
        // order are the segments (jr, kappa chunk) in turn.
        auto test = [&](int jr, int k, int32_t *v_out) {
            if (k >= nk)
                return false;
            const int at = (jr + 1) * W + k + 1;
            const int32_t *m = mid + at;
            const int32_t v = m[0];
            int32_t before = max(max3i(m[-W - 1], m[-W], m[-W + 1]), m[-1]);
            int32_t after = max(max3i(m[W - 1], m[W], m[W + 1]), m[1]);
            if (has_lo) {
                const int32_t *q = lo + at;
                before = max(before, max3i(max3i(q[-W - 1], q[-W], q[-W + 1]), max3i(q[-1], q[0], q[1]),
                                           max3i(q[W - 1], q[W], q[W + 1])));
            }
            if (has_hi) {
                const int32_t *q = hi + at;
                after = max(after, max3i(max3i(q[-W - 1], q[-W], q[-W + 1]), max3i(q[-1], q[0], q[1]),
                                         max3i(q[W - 1], q[W], q[W + 1])));
            }
            *v_out = v;
            return v >= thr && v > before && v >= after;
        };
        // pass 1: survivor lanes per segment and wavefront (every lane writes
        // the same mask).  One kappa chunk per row (n_kappa <= the block
        // size) unrolls over the rows, so their LDS reads overlap.
        if (nk <= kPeakThreads) {
#pragma unroll
            for (int jr = 0; jr < kPeakRows; ++jr) {
                if (jr < rows_here) {
                    int32_t v;
                    const bool keep = test(jr, tid, &v);
                    sc.seg_mask[jr][wave] = __ballot(keep);
                }
            }
        } else {
            for (int jr = 0, s = 0; jr < rows_here; ++jr) {
                for (int k0 = 0; k0 < nk; k0 += kPeakThreads, ++s) {
                    int32_t v;
                    const bool keep = test(jr, k0 + tid, &v);
                    sc.seg_mask[s][wave] = __ballot(keep);
                }
            }
        }
        // Slice l+2 goes into the slot slice l-2 held (read last in the
        // previous step); stored now, before this step's candidate stores
        // queue behind its loads.
        if (next2) {
            if (overlap) {
                commit_first(l + 2);
                pad(l + 2);
            } else {
                load(l + 2);
            }
        }
        lds_barrier();
        // pass 2: write survivors in cell order
        Cand *out = a.w.s0.stage + (static_cast<int64_t>(e) * a.w.s0.n_blocks0 + l * bps + rb) * a.w.s0.cap0;
        const int64_t cell_base = (static_cast<int64_t>(l) * g.n_phi + j0) * nk;
        uint32_t kmin = 0xffffffffu, kmax = 0u;
        int base = 0;
        for (int jr = 0, s = 0; jr < rows_here; ++jr) {
            for (int k0 = 0; k0 < nk; k0 += kPeakThreads, ++s) {
                int pre = 0, total = 0;
#pragma unroll
                for (int w2 = 0; w2 < kPeakWaves; ++w2) {
                    const int c = __popcll(sc.seg_mask[s][w2]);
                    pre += w2 < wave ? c : 0;
                    total += c;
                }
                const uint64_t msk = sc.seg_mask[s][wave];
                const bool keep = (msk >> lane) & 1u;
                if (keep) {
                    const int k = k0 + tid;
                    const int32_t v = mid[(jr + 1) * W + k + 1];
                    out[base + pre + rank_below(msk)] = Cand{v, static_cast<int32_t>(cell_base + jr * nk + k)};
                    const uint32_t key = sort_key(v);
                    atomicAdd(&sc.hist[key & 0xffu], 1u);
                    kmin = min(kmin, key);
                    kmax = max(kmax, key);
                }
                base += total;
            }
        }
        kmin = wave_min_u32(kmin);
        kmax = wave_max_u32(kmax);
        if (lane == 0) {
            sc.red_min[wave] = kmin;
            sc.red_max[wave] = kmax;
        }
        lds_barrier();
        uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
        for (int w2 = 0; w2 < kPeakWaves; ++w2) {
            mn = min(mn, sc.red_min[w2]);
            mx = max(mx, sc.red_max[w2]);
        }
        if (tid == 0) {
            a.w.s0.cnt0[static_cast<int64_t>(e) * a.w.s0.n_blocks0 + l * bps + rb] = base;
            if (base > 0) {
                atomicMin(&a.w.state[e].key_min, mn);
                atomicMax(&a.w.state[e].key_max, mx);
            }
        }
        const int chunk = (l * bps + rb) / a.w.s0.cb;
        uint32_t *hrow = a.w.hist + (static_cast<int64_t>(e) * a.w.hist_chunks + chunk) * kDigits;
        for (int i = tid; i < kDigits; i += kPeakThreads) {
            if (a.w.s0.cb == 1)
                hrow[i] = sc.hist[i];
            else if (sc.hist[i])
                atomicAdd(&hrow[i], sc.hist[i]);
        }
        lds_barrier();   // the histogram and the ring are reused
    }
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
            lds_barrier();
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
            lds_barrier();
            if (valid) {
                uint32_t pre = run[digit];
                for (int w2 = 0; w2 < wave; ++w2)
                    pre += wcnt[w2][digit];
                const int64_t pos = static_cast<int64_t>(pre) + rank;
                if (pos < limit)
                    dst[pos] = cd;
            }
            lds_barrier();
            for (int dd = t; dd < kDigits; dd += kSortThreads) {
                uint32_t add = 0;
                for (int w2 = 0; w2 < kWaves; ++w2)
                    add += wcnt[w2][dd];
                run[dd] += add;
            }
            lds_barrier();
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
    if (kPeakRows * ((g.n_kappa + kPeakThreads - 1) / kPeakThreads) > kMaxSegs)
        return hipErrorInvalidValue;   // more kappa bins than one band's survivor bookkeeping holds
    const size_t lds = (static_cast<size_t>(g.n_d0 > 1 ? 4 : 1) * kHaloRows * (g.n_kappa + 2) + 2 * kPeakThreads) *
                       sizeof(int32_t);
    const void *fn = u16 ? reinterpret_cast<const void *>(peak_kernel<true>)
                         : reinterpret_cast<const void *>(peak_kernel<false>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    const int32_t slice_chunks = (g.n_d0 + kPeakSlices - 1) / kPeakSlices;
    dim3 grid(static_cast<unsigned>(a.blocks_per_slice * slice_chunks), static_cast<unsigned>(n_events));
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
