// Device helpers shared by the peak search kernels: wavefront reductions and
// the publication of an ordered staging list for the candidate sort.
#pragma once

#include "hough_impl.h"

namespace hough {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the wavefront; the kernels here
// exchange data between threads through LDS alone (their global results are
// read by later kernels), so waiting for global memory at each barrier would
// only expose its latency -- and cancel the loads issued ahead of time.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// Shared-memory scratch of one ordered compaction.
template <int NT>
struct CompactScratch {
    uint32_t hist[kDigits];
    int32_t wave_cnt[NT / 64];
    uint32_t red_min[NT / 64];
    uint32_t red_max[NT / 64];
};

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
