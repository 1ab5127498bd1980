// Peak search and candidate ordering for gfx950.
//
// Section 3: after voting, local maxima of the parameter space are the track
// candidates.  Each wavefront owns a strip of one d0 slice -- whole phi0 rows
// when a row is at most 64 lanes of 4 dwords, else 64 lanes' worth of one
// row -- and walks kPeakSlices consecutive d0 slices of it.  A lane holds 4
// consecutive dwords of a row (8 uint16 or 4 int32 cells) and loads them, for
// rows j-1, j, j+1 (phi0 wraps), straight from memory, one slice ahead of the
// test; kappa neighbours across lanes come from lane shifts (from memory at a
// wavefront boundary inside a row), and cells outside the kappa or d0 range
// count as INT_MIN, which never blocks a cell.
//
// The asymmetric 3x3(x3) test of hough.h is separable: with A = the maximum of
// a cell and its two kappa neighbours in one row and B = the maximum of A over
// rows j-1, j, j+1 (the 3x3 square of one slice), a cell passes when it
// reaches the threshold, exceeds max(B of slice l-1, A of row j-1, its left
// neighbour) and reaches max(B of slice l+1, A of row j+1, its right
// neighbour).  B of each slice is computed once and kept in registers for the
// two slices that use it, so a cell costs about ten VALU operations and no
// LDS reads.
//
// Four wavefronts form a block; the survivors of one block and slice are one
// staging list in ascending cell order (lane order within a wavefront, then
// wavefront order), placed after one LDS exchange of wavefront counts.  Their
// first-digit histogram is counted in LDS and the event's key range is
// published once per block.
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
#include <algorithm>
#include <climits>

#include "hough_impl.h"
#include "peak_tile.h"

namespace hough {
namespace {

constexpr int kPeakThreads = 256;
constexpr int kPeakWaves = kPeakThreads / 64;
constexpr int kPeakSlices = 8;     // d0 slices walked per block (at most)
constexpr size_t kPeakLdsBudget = 40 * 1024;   // staged lists and histograms per block

// Strips of one d0 slice.  A phi0 row is lpr lanes of 4 dwords (the last lane
// of a row may hold fewer).  lpr <= 64: a wavefront holds rpw = 64 / lpr whole
// rows; lpr > 64: a row is wpr wavefronts.
struct PeakLayout {
    int32_t lpr;
    int32_t rpw;             // 0 when lpr > 64
    int32_t wpr;             // 0 when lpr <= 64
    int32_t strips;          // wavefront strips per slice
    int32_t bands;           // blocks per slice (kPeakWaves consecutive strips)
    int32_t rows_per_band;   // phi0 rows one band can touch
};

PeakLayout peak_layout(const GridArgs &g) {
    PeakLayout p{};
    p.lpr = (g.row_dwords + 3) / 4;
    if (p.lpr <= 64) {
        p.rpw = 64 / p.lpr;
        p.strips = (g.n_phi + p.rpw - 1) / p.rpw;
        p.rows_per_band = kPeakWaves * p.rpw;
    } else {
        p.wpr = (p.lpr + 63) / 64;
        p.strips = g.n_phi * p.wpr;
        if (p.wpr % kPeakWaves == 0)
            p.rows_per_band = 1;
        else if (kPeakWaves % p.wpr == 0)
            p.rows_per_band = kPeakWaves / p.wpr;
        else
            p.rows_per_band = (kPeakWaves + p.wpr - 1) / p.wpr + 1;
    }
    p.bands = (p.strips + kPeakWaves - 1) / kPeakWaves;
    return p;
}

struct PeakArgs {
    GridArgs g;
    const uint32_t *acc;     // dwords, events back to back
    int32_t threshold;
    int32_t lpr, rpw, wpr, bands;
    int32_t slices;          // d0 slices walked per block
    SortWork w;
};

__device__ __forceinline__ int32_t max3i(int32_t a, int32_t b, int32_t c) { return max(max(a, b), c); }

// One slice as seen by a lane: its cells of row j with their outer kappa
// neighbours, A of rows j-1 and j+1, and B.
template <int CPL>
struct SliceView {
    int32_t v[CPL];
    int32_t left, right;
    int32_t au[CPL], ad[CPL], b[CPL];
};

template <bool U16, bool VEC>
__global__ __launch_bounds__(kPeakThreads) void peak_kernel(PeakArgs a) {
    constexpr int CPL = U16 ? 8 : 4;
    // LDS: per walked slice a 256-bin histogram, a count and a candidate list
    // of cap0 entries; global stores wait until the walk is done, so the only
    // memory operations in the walk are the slice loads.
    extern __shared__ uint32_t dyn[];
    __shared__ int32_t wcnt[2][kPeakWaves];
    __shared__ uint32_t wmin[2][kPeakWaves];
    __shared__ uint32_t wmax[2][kPeakWaves];
    __shared__ int32_t scnt[kPeakSlices];
    const int S = a.slices;
    const int cap0 = a.w.s0.cap0;
    uint32_t *const hist = dyn;                                          // [S][kDigits]
    Cand *const cands = reinterpret_cast<Cand *>(dyn + S * kDigits);     // [S][cap0]

    const GridArgs &g = a.g;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int e = blockIdx.y;
    if (a.w.n_events_dev && e >= *a.w.n_events_dev)
        return;
    const int band = blockIdx.x % a.bands;
    const int l0 = (blockIdx.x / a.bands) * a.slices;
    const int l1 = min(g.n_d0, l0 + a.slices);
    const int n_phi = g.n_phi;
    const int nk = g.n_kappa;
    const int rd = g.row_dwords;
    const int lpr = a.lpr;
    const int strip = band * kPeakWaves + wave;
    int j, ri;
    bool active;
    if (a.rpw > 0) {
        const int ro = lane / lpr;
        ri = lane - ro * lpr;
        j = strip * a.rpw + ro;
        active = ro < a.rpw && j < n_phi;
    } else {
        j = strip / a.wpr;
        ri = (strip - j * a.wpr) * 64 + lane;
        active = j < n_phi && ri < lpr;
    }
    const int dw0 = ri * 4;
    const int ndw = active ? min(4, rd - dw0) : 0;
    const int jj = active ? j : 0;
    const int jm = jj == 0 ? n_phi - 1 : jj - 1;
    const int jp = jj + 1 == n_phi ? 0 : jj + 1;
    const int roff[3] = {jm * rd + dw0, jj * rd + dw0, jp * rd + dw0};
    const bool row_first = ri == 0;
    const bool row_last = ri == lpr - 1;
    // neighbour dwords in another wavefront of the same row
    const bool left_mem = active && !row_first && a.wpr > 0 && lane == 0;
    const bool right_mem = active && !row_last && a.wpr > 0 && lane == 63;
    const uint32_t *acc_e = a.acc + static_cast<int64_t>(e) * g.acc_dwords;
    const int64_t plane = static_cast<int64_t>(n_phi) * rd;

    auto load = [&](int ll, uint32_t (&r)[3][4], uint32_t (&x)[3][2]) {
        const uint32_t *p = acc_e + static_cast<int64_t>(ll) * plane;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if constexpr (VEC) {
                uint4 d = make_uint4(0u, 0u, 0u, 0u);
                if (active)
                    d = *reinterpret_cast<const uint4 *>(p + roff[q]);
                r[q][0] = d.x;
                r[q][1] = d.y;
                r[q][2] = d.z;
                r[q][3] = d.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    r[q][k] = k < ndw ? p[roff[q] + k] : 0u;
            }
            x[q][0] = left_mem ? p[roff[q] - 1] : 0u;
            x[q][1] = right_mem ? p[roff[q] + 4] : 0u;
        }
    };
    // cells of one row with the kappa maxima A; returns the outer neighbours
    auto row = [&](const uint32_t (&d)[4], const uint32_t (&x)[2], int32_t (&c)[CPL], int32_t (&m)[CPL],
                   int32_t &left, int32_t &right) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (U16) {
                c[2 * k] = k < ndw ? static_cast<int32_t>(d[k] & 0xffffu) : INT_MIN;
                c[2 * k + 1] = k < ndw ? static_cast<int32_t>(d[k] >> 16) : INT_MIN;
            } else {
                c[k] = k < ndw ? static_cast<int32_t>(d[k]) : INT_MIN;
            }
        }
        left = __shfl_up(c[CPL - 1], 1);
        right = __shfl_down(c[0], 1);
        if (row_first)
            left = INT_MIN;
        else if (left_mem)
            left = U16 ? static_cast<int32_t>(x[0] >> 16) : static_cast<int32_t>(x[0]);
        if (row_last)
            right = INT_MIN;
        else if (right_mem)
            right = U16 ? static_cast<int32_t>(x[1] & 0xffffu) : static_cast<int32_t>(x[1]);
#pragma unroll
        for (int i = 0; i < CPL; ++i)
            m[i] = max3i(i == 0 ? left : c[i - 1], c[i], i == CPL - 1 ? right : c[i + 1]);
    };
    auto view = [&](const uint32_t (&r)[3][4], const uint32_t (&x)[3][2], SliceView<CPL> &s) {
        int32_t cu[CPL], cd[CPL], am[CPL];
        int32_t lu, ru, ld, rdn;
        row(r[0], x[0], cu, s.au, lu, ru);
        row(r[1], x[1], s.v, am, s.left, s.right);
        row(r[2], x[2], cd, s.ad, ld, rdn);
#pragma unroll
        for (int i = 0; i < CPL; ++i)
            s.b[i] = max3i(s.au[i], am[i], s.ad[i]);
    };

    uint32_t raw[3][4], rx[3][2];
    int32_t pb[CPL];                // B of slice l - 1
    SliceView<CPL> cur;
    {
        uint32_t r0[3][4], x0[3][2], r1[3][4], x1[3][2];
        const bool has_prev = l0 > 0;
        if (has_prev)
            load(l0 - 1, r0, x0);
        load(l0, r1, x1);
        if (l0 + 1 < g.n_d0)
            load(l0 + 1, raw, rx);
        if (has_prev) {
            SliceView<CPL> p;
            view(r0, x0, p);
#pragma unroll
            for (int i = 0; i < CPL; ++i)
                pb[i] = p.b[i];
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
                pb[i] = INT_MIN;
        }
        view(r1, x1, cur);
    }
    for (int i = tid; i < S * kDigits; i += kPeakThreads)
        hist[i] = 0u;
    lds_barrier();

    const int32_t thr = a.threshold;
    uint32_t run_min = 0xffffffffu, run_max = 0u;
    for (int l = l0; l < l1; ++l) {
        const int par = (l - l0) & 1;
        SliceView<CPL> nxt;
        if (l + 1 < g.n_d0) {
            view(raw, rx, nxt);
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
                nxt.b[i] = INT_MIN;
        }
        if (l + 2 < g.n_d0 && l + 2 <= l1)
            load(l + 2, raw, rx);

        uint32_t mask = 0u;
        int32_t vmax = INT_MIN, vmin = INT_MAX;
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            const int32_t v = cur.v[i];
            const int32_t before = max3i(pb[i], cur.au[i], i == 0 ? cur.left : cur.v[i - 1]);
            const int32_t after = max3i(nxt.b[i], cur.ad[i], i == CPL - 1 ? cur.right : cur.v[i + 1]);
            const bool keep = v >= thr && v > before && v >= after;
            mask |= keep ? (1u << i) : 0u;
            vmax = keep ? max(vmax, v) : vmax;
            vmin = keep ? min(vmin, v) : vmin;
        }
        // at most CPL / 2 survivors per lane: kappa neighbours cannot both pass
        const int s = l - l0;
        const int n = __popc(mask);
        const uint64_t b0 = __ballot(n & 1);
        const uint64_t b1 = __ballot(n & 2);
        const uint64_t b2 = __ballot(n & 4);
        const int pre = rank_below(b0) + 2 * rank_below(b1) + 4 * rank_below(b2);
        const int tot = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
        // (every loop over a lane's cells is unrolled with constant indices:
        // a register array indexed at run time costs a wait on the loads in
        // flight)
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            if ((mask >> i) & 1u)
                atomicAdd(&hist[s * kDigits + (sort_key(cur.v[i]) & 0xffu)], 1u);
        }
        const uint32_t kmn = wave_min_u32(mask ? sort_key(vmax) : 0xffffffffu);
        const uint32_t kmx = wave_max_u32(mask ? sort_key(vmin) : 0u);
        if (lane == 0) {
            wcnt[par][wave] = tot;
            wmin[par][wave] = kmn;
            wmax[par][wave] = kmx;
        }
        lds_barrier();
        int base = 0, all = 0;
        uint32_t bmin = 0xffffffffu, bmax = 0u;
#pragma unroll
        for (int w2 = 0; w2 < kPeakWaves; ++w2) {
            const int c = wcnt[par][w2];
            base += w2 < wave ? c : 0;
            all += c;
            bmin = min(bmin, wmin[par][w2]);
            bmax = max(bmax, wmax[par][w2]);
        }
        // A list never holds more than cap0 survivors (an independent set of
        // the king's graph); the clamps only keep memory safe.
        if (mask) {
            Cand *out = cands + s * cap0;
            const int32_t cell0 = (l * n_phi + j) * nk + ri * CPL;
            int m = base + pre;
#pragma unroll
            for (int i = 0; i < CPL; ++i) {
                if ((mask >> i) & 1u) {
                    if (m < cap0)
                        out[m] = Cand{cur.v[i], cell0 + i};
                    ++m;
                }
            }
        }
        if (tid == 0) {
            scnt[s] = min(all, cap0);
            run_min = min(run_min, bmin);
            run_max = max(run_max, bmax);
        }
#pragma unroll
        for (int i = 0; i < CPL; ++i)
            pb[i] = cur.b[i];
        cur = nxt;
    }
    lds_barrier();
    // write out the walk: counts, lists and first-digit histograms
    const int n_s = l1 - l0;
    const int64_t n_blocks0 = a.w.s0.n_blocks0;
    for (int s = 0; s < n_s; ++s) {
        const int l = l0 + s;
        const int64_t list = static_cast<int64_t>(e) * n_blocks0 + static_cast<int64_t>(l) * a.bands + band;
        const int c = scnt[s];
        if (tid == 0)
            a.w.s0.cnt0[list] = c;
        Cand *dst = a.w.s0.stage + list * cap0;
        for (int i = tid; i < c; i += kPeakThreads)
            dst[i] = cands[s * cap0 + i];
        const int chunk = (l * a.bands + band) / a.w.s0.cb;
        uint32_t *hrow = a.w.hist + (static_cast<int64_t>(e) * a.w.hist_chunks + chunk) * kDigits;
        const uint32_t h = hist[s * kDigits + tid];
        if (a.w.s0.cb == 1)
            hrow[tid] = h;
        else if (h)
            atomicAdd(&hrow[tid], h);
    }
    if (tid == 0 && run_min <= run_max) {
        atomicMin(&a.w.state[e].key_min, run_min);
        atomicMax(&a.w.state[e].key_max, run_max);
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

// Packed lists (batch): event e's stored list, min(n_found, its capacity)
// candidates, starts where event e - 1's ends, so a batch's lists fill
// out[0, cand_start[n_events]) and one copy moves them all.  One workgroup,
// after the pass-0 scan has fixed every n_found and before any scatter writes
// the output; each thread sums a run of consecutive events, and a scan over
// the threads turns the sums into offsets.
constexpr int kPackThreads = 1024;

__global__ __launch_bounds__(kPackThreads) void pack_kernel(SortWork w, int32_t max_events) {
    __shared__ int64_t part[kPackThreads];
    const int n = w.n_events_dev ? min(*w.n_events_dev, max_events) : max_events;
    const int t = threadIdx.x;
    const int per = (n + kPackThreads - 1) / kPackThreads;
    const int begin = min(n, t * per);
    const int end = min(n, begin + per);
    int64_t sum = 0;
    for (int e = begin; e < end; ++e)
        sum += min(w.state[e].n_found, w.desc[e].cand_cap);
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < kPackThreads; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int e = begin; e < end; ++e) {
        w.cand_start[e] = run;
        run += min(w.state[e].n_found, w.desc[e].cand_cap);
    }
    if (t == kPackThreads - 1)
        w.cand_start[n] = part[t];
}

// Stable scatter of one chunk by the digit of this pass.  A round takes up to
// 2,048 consecutive elements, split into one run per wavefront (a
// multiple of 64, at most 64 * kSortPer, shorter when the list is short so
// that every wavefront has a share), lane by lane in sub-blocks of 64, all
// loads issued first.  Each wavefront
// ranks its elements within their digit on its own (a running count per digit
// in LDS, updated by the first lane of each digit of a sub-block); one
// barrier, a prefix over wavefronts per digit, a second barrier, and every
// element goes to run[digit] + its wavefront's prefix + its rank.
constexpr int kSortPer = 8;

__global__ __launch_bounds__(kSortThreads) void scatter_kernel(SortWork w, int pass) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t run[kDigits];
    __shared__ uint32_t wcnt[kWaves][kDigits];
    __shared__ uint32_t wpre[kWaves][kDigits];
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
            dst = reinterpret_cast<Cand *>(w.out) + (w.cand_start ? w.cand_start[e] : w.desc[e].cand_begin);
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
    const int lane = t & 63;
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
        for (int b0 = 0; b0 < count;) {
            const int rem = count - b0;
            const int seg = min(64 * kSortPer, ((rem + kWaves - 1) / kWaves + 63) & ~63);
            const int subs = seg >> 6;
            // this wavefront's elements of the round, loaded at once
            const int base = b0 + wave * seg + lane;
            Cand cd[kSortPer];
#pragma unroll
            for (int k = 0; k < kSortPer; ++k) {
                const int i = base + 64 * k;
                cd[k] = (k < subs && i < count) ? src[i] : Cand{0, 0};
            }
            for (int d = lane; d < kDigits; d += 64)
                wcnt[wave][d] = 0u;
            __builtin_amdgcn_wave_barrier();
            uint32_t digit[kSortPer] = {};
            uint32_t rank[kSortPer] = {};
#pragma unroll
            for (int k = 0; k < kSortPer; ++k) {
                if (k >= subs)
                    break;                      // wave-uniform: short runs stop early
                const bool valid = base + 64 * k < count;
                digit[k] = valid ? (sort_key(cd[k].votes) >> shift) & 0xffu : 0u;
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int bit = 0; bit < 8; ++bit) {
                    const bool set = (digit[k] >> bit) & 1u;
                    const uint64_t bb = __ballot(set);
                    peers &= set ? bb : ~bb;
                }
                const int r = rank_below(peers);
                const uint32_t before = valid ? wcnt[wave][digit[k]] : 0u;
                __builtin_amdgcn_wave_barrier();
                if (valid && r == 0)
                    wcnt[wave][digit[k]] = before + static_cast<uint32_t>(__popcll(peers));
                __builtin_amdgcn_wave_barrier();
                rank[k] = valid ? before + static_cast<uint32_t>(r) : 0u;
            }
            lds_barrier();
            // per digit: the prefix over wavefronts on top of run, and the new run
            for (int d = t; d < kDigits; d += kSortThreads) {
                uint32_t acc = run[d];
#pragma unroll
                for (int w2 = 0; w2 < kWaves; ++w2) {
                    wpre[w2][d] = acc;
                    acc += wcnt[w2][d];
                }
                run[d] = acc;
            }
            lds_barrier();
#pragma unroll
            for (int k = 0; k < kSortPer; ++k) {
                if (k < subs && base + 64 * k < count) {
                    const int64_t pos = static_cast<int64_t>(wpre[wave][digit[k]]) + rank[k];
                    if (pos < limit)
                        dst[pos] = cd[k];
                }
            }
            b0 += kWaves * seg;
        }
    }
}

}  // namespace

int32_t peak_blocks_per_event(const GridArgs &g) {
    return g.n_d0 * peak_layout(g).bands;
}

int32_t peak_block_cap(const GridArgs &g) {
    // Survivors of one block and slice form an independent set of the king's
    // graph on the rows it touches: at most ceil(rows/2) * ceil(n_kappa/2).
    return ((peak_layout(g).rows_per_band + 1) / 2) * ((g.n_kappa + 1) / 2);
}

int32_t peak_blocks_per_chunk(const GridArgs &g) {
    // At most 256 first-pass chunks per event keeps the offset scan short.
    const int32_t blocks = peak_blocks_per_event(g);
    return (blocks + 255) / 256;
}

hipError_t launch_peaks(const GridArgs &g, bool u16, const uint32_t *acc, int32_t n_events,
                        int32_t threshold, const SortWork &w, hipStream_t stream) {
    const PeakLayout lay = peak_layout(g);
    PeakArgs a{};
    a.g = g;
    a.acc = acc;
    a.threshold = threshold;
    a.lpr = lay.lpr;
    a.rpw = lay.rpw;
    a.wpr = lay.wpr;
    a.bands = lay.bands;
    a.w = w;
    if (w.s0.cb > 1) {
        // blocks add into shared first-pass histogram rows
        hipError_t e = launch_zero(w.hist, static_cast<int64_t>(n_events) * w.hist_chunks * kDigits, stream);
        if (e != hipSuccess)
            return e;
    }
    // 16-byte row loads when every row starts on a 16-byte boundary
    const bool vec = g.row_dwords % 4 == 0 && (reinterpret_cast<uintptr_t>(acc) & 15u) == 0;
    // slices per block: as many as kPeakLdsBudget of staged lists allows (a
    // list of a grid the vote accepts, n_kappa <= 1200 or so, is a few KB)
    const size_t per_slice = kDigits * sizeof(uint32_t) + static_cast<size_t>(w.s0.cap0) * sizeof(Cand);
    if (per_slice > kPeakLdsBudget)
        return hipErrorInvalidValue;
    a.slices = static_cast<int32_t>(std::min<size_t>(kPeakSlices, kPeakLdsBudget / per_slice));
    const size_t lds = a.slices * per_slice;
    const int32_t slice_chunks = (g.n_d0 + a.slices - 1) / a.slices;
    dim3 grid(static_cast<unsigned>(lay.bands * slice_chunks), static_cast<unsigned>(n_events));
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(kPeakThreads), lds, stream, a);
    };
    if (u16)
        vec ? go(peak_kernel<true, true>) : go(peak_kernel<true, false>);
    else
        vec ? go(peak_kernel<false, true>) : go(peak_kernel<false, false>);
    return hipGetLastError();
}

hipError_t launch_sort(const SortWork &w, int32_t n_events, hipStream_t stream) {
    // one pass per 8-bit digit that can differ (at least one: it places the lists)
    int max_passes = 1;
    while (max_passes < kMaxPasses && (w.key_mask >> (8 * max_passes)) != 0u)
        ++max_passes;
    const unsigned later_chunks = static_cast<unsigned>((w.bound + kSortChunk - 1) / kSortChunk);
    const unsigned first_chunks = static_cast<unsigned>((w.s0.n_blocks0 + w.s0.cb - 1) / w.s0.cb);
    for (int pass = 0; pass < max_passes; ++pass) {
        if (pass > 0)
            hipLaunchKernelGGL(hist_kernel, dim3(later_chunks, n_events), dim3(kSortThreads), 0, stream, w, pass);
        hipLaunchKernelGGL(scan_kernel, dim3(n_events), dim3(kScanThreads), 0, stream, w, pass);
        if (pass == 0 && w.cand_start && w.desc)
            hipLaunchKernelGGL(pack_kernel, dim3(1), dim3(kPackThreads), 0, stream, w, n_events);
        const unsigned chunks = pass == 0 ? first_chunks : later_chunks;
        hipLaunchKernelGGL(scatter_kernel, dim3(chunks, n_events), dim3(kSortThreads), 0, stream, w, pass);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace hough
