// Device helpers shared by the peak search kernels: the asymmetric local
// maximum test and ordered compaction of survivors into a staging list.
#pragma once

#include "hough_impl.h"

namespace hough {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ int rank_below(uint64_t mask) {
    return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u)));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = min(v, static_cast<uint32_t>(__shfl_xor(v, off, 64)));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = max(v, static_cast<uint32_t>(__shfl_xor(v, off, 64)));
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Shared-memory scratch of one compaction pass.
template <int NT>
struct CompactScratch {
    uint32_t hist[kDigits];
    int32_t wave_cnt[NT / 64];
    uint32_t red_min[NT / 64];
    uint32_t red_max[NT / 64];
};

// Local-maximum test of a 2D cell (phi0 row r of an LDS tile whose rows
// r-1 and r+1 are present, kappa bin k): negative offsets need v > w,
// positive ones v >= w; kappa neighbours outside [0, nk) are ignored.
__device__ __forceinline__ bool is_peak_2d(const int32_t *row, int stride, int nk, int k, int32_t v) {
    const int32_t *up = row - stride;
    const int32_t *dn = row + stride;
    bool ok = true;
    if (k > 0)
        ok = ok && v > up[k - 1] && v >= dn[k - 1] && v > row[k - 1];
    ok = ok && v > up[k] && v >= dn[k];
    if (k + 1 < nk)
        ok = ok && v > up[k + 1] && v >= dn[k + 1] && v >= row[k + 1];
    return ok;
}

// Scan `n_cells` cells of an LDS tile in order, keep those `test` accepts and
// append them, in that order, to `out`.  Also accumulates the lowest sort
// digit histogram in sc.hist (zeroed by the caller) and the smallest and
// largest sort key.  Returns the number kept (uniform across the block).
// `test(idx, &v, &cell)` evaluates cell idx.
template <int NT, typename Test>
__device__ int compact_ordered(int n_cells, Test test, Cand *out, CompactScratch<NT> &sc, uint32_t *kmin_out,
                               uint32_t *kmax_out) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    uint32_t kmin = 0xffffffffu, kmax = 0u;
    int base = 0;
    for (int r0 = 0; r0 < n_cells; r0 += NT) {
        const int idx = r0 + tid;
        int32_t v = 0, cell = 0;
        const bool keep = idx < n_cells && test(idx, &v, &cell);
        const uint64_t m = __ballot(keep);
        if (lane_id() == 0)
            sc.wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int pre = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            const int c = sc.wave_cnt[w];
            pre += w < wave ? c : 0;
            total += c;
        }
        if (keep) {
            out[base + pre + rank_below(m)] = Cand{v, cell};
            const uint32_t key = sort_key(v);
            atomicAdd(&sc.hist[key & 0xffu], 1u);
            kmin = min(kmin, key);
            kmax = max(kmax, key);
        }
        base += total;
        __syncthreads();
    }
    kmin = wave_min_u32(kmin);
    kmax = wave_max_u32(kmax);
    if (lane_id() == 0) {
        sc.red_min[wave] = kmin;
        sc.red_max[wave] = kmax;
    }
    __syncthreads();
    uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        mn = min(mn, sc.red_min[w]);
        mx = max(mx, sc.red_max[w]);
    }
    *kmin_out = mn;
    *kmax_out = mx;
    return base;
}

// Publish one staging list (block): its count, its key range and its digit
// histogram.  With one list per first-pass chunk the histogram row is
// written; with several, the lists add into a row the caller zeroed.
template <int NT>
__device__ void publish_block(const SortWork &w, int e, int block, int count, CompactScratch<NT> &sc,
                              uint32_t kmin, uint32_t kmax) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        w.s0.cnt0[static_cast<int64_t>(e) * w.s0.n_blocks0 + block] = count;
        if (count > 0) {
            atomicMin(&w.state[e].key_min, kmin);
            atomicMax(&w.state[e].key_max, kmax);
        }
    }
    const int chunk = block / w.s0.cb;
    uint32_t *hrow = w.hist + (static_cast<int64_t>(e) * w.hist_chunks + chunk) * kDigits;
    if (w.s0.cb == 1) {
        for (int i = tid; i < kDigits; i += NT)
            hrow[i] = sc.hist[i];
    } else {
        for (int i = tid; i < kDigits; i += NT) {
            const uint32_t v = sc.hist[i];
            if (v)
                atomicAdd(&hrow[i], v);
        }
    }
}

}  // namespace hough
