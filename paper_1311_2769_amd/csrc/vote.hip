// Hough vote kernels for gfx950.
//
// Section 3: every hypothesis starts with zero votes and every hit adds one
// vote to each hypothesis it lies on; Section 4: the work for each hit is
// independent of the others.  The accumulator is split into tiles of
// consecutive phi0 rows of one d0 slice.  A workgroup owns one tile as a
// private LDS accumulator, streams every hit of the event through it (each
// lane evaluates its own phi0 row, so a wave covers 64 rows of one hit or
// 64/rows hits of a narrower tile) and flushes the finished tile to HBM with
// coalesced stores: no global atomics on the accumulator.  The vote count is
// reduced per wavefront and added once per workgroup.
//
// Arithmetic is the fp32 definition in hough.h, op for op; this file is
// compiled with -ffp-contract=off and the default correctly rounded divide.
// For the 2D grid (d0 == +0) the numerator 2*(u - 0) equals 2*u and the
// denominator (r2 - 0*u) + 0*0 equals r2 for every finite u, and both forms
// give NaN or an out-of-range kf otherwise, so the 2D kernels use 2*u / r2.
//
// uint16 accumulators are packed two cells per dword in LDS (even kappa bin in
// the low half): a vote adds 1 or 0x10000 with one 32-bit LDS atomic.  The low
// half can never carry into the high half because a cell receives at most one
// vote per hit and u16 events hold at most 65535 hits.
#pragma clang fp contract(off)

#include "hough_impl.h"

namespace hough {
namespace {

struct VoteKernelArgs {
    GridArgs g;
    const float *x;
    const float *y;
    int32_t n_hits;             // single event
    int32_t split;              // single event: hit chunks per tile
    int32_t tiles_per_slice;
    int32_t lds_stride;         // dwords per LDS row
    const EventDesc *desc;      // batch: per-event hit ranges
    const WorkItem *items;      // batch: tile list, or nullptr for a single event
    const int32_t *n_items;     // batch: live item count (device)
    int32_t *work_counter;      // batch, persistent: next item to take
    uint32_t *acc;              // dwords
    unsigned long long *n_votes;
};

__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Vote hits [h_begin, h_end) into the tile (l, j0 .. j0+ROWS) and flush it.
template <bool U16, bool D3, int RL, int RPT, int NT>
__device__ void vote_tile(const VoteKernelArgs &a, int64_t h_begin, int64_t h_end, int l, int j0,
                          uint32_t *__restrict__ acc_event, bool atomic_flush,
                          unsigned long long *n_votes, uint32_t *lds, uint32_t *red) {
    constexpr int ROWS = RL * RPT;
    constexpr int HSTEP = NT / RL;
    const GridArgs &g = a.g;
    const int tid = threadIdx.x;
    const int stride = a.lds_stride;
    const int rows_here = min(ROWS, g.n_phi - j0);

    for (int i = tid; i < rows_here * stride; i += NT)
        lds[i] = 0u;
    __syncthreads();

    const int lane_row = tid % RL;
    int hslot = tid / RL;
    if constexpr (RL == 64)
        hslot = __builtin_amdgcn_readfirstlane(hslot);   // one hit per wavefront
    float c[RPT], s[RPT];
    int rowoff[RPT];
    bool live[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int jr = lane_row + r * RL;
        live[r] = jr < rows_here;
        const int j = j0 + (live[r] ? jr : 0);
        c[r] = g.cos_phi[j];
        s[r] = g.sin_phi[j];
        rowoff[r] = jr * stride;
    }
    const float d = D3 ? g.d0[l] : 0.0f;
    const float d2 = 2.0f * d;
    const float dd = d * d;
    const float kmin = g.kappa_min;
    const float kscale = g.kappa_scale;
    const float nkf = static_cast<float>(g.n_kappa);

    const float *__restrict__ xs = a.x;
    const float *__restrict__ ys = a.y;
    uint32_t votes = 0;
    for (int64_t h = h_begin + hslot; h < h_end; h += HSTEP) {
        const float xh = xs[h];
        const float yh = ys[h];
        const float r2 = xh * xh + yh * yh;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const float u = yh * c[r] - xh * s[r];
            float kappa;
            if constexpr (D3) {
                const float num = 2.0f * (u - d);
                const float den = (r2 - d2 * u) + dd;
                kappa = num / den;
            } else {
                kappa = (2.0f * u) / r2;
            }
            const float kf = (kappa - kmin) * kscale;
            if (live[r] && kf >= 0.0f && kf < nkf) {
                const int k = static_cast<int>(kf);
                if constexpr (U16)
                    lds_add(&lds[rowoff[r] + (k >> 1)], (k & 1) ? 0x10000u : 1u);
                else
                    lds_add(&lds[rowoff[r] + k], 1u);
                ++votes;
            }
        }
    }
    __syncthreads();

    // Flush the tile: rows are contiguous in the global accumulator.
    const int rd = g.row_dwords;
    uint32_t *dst = acc_event + (static_cast<int64_t>(l) * g.n_phi + j0) * rd;
    if (!atomic_flush) {
        for (int rr = 0; rr < rows_here; ++rr)
            for (int w = tid; w < rd; w += NT)
                dst[static_cast<int64_t>(rr) * rd + w] = lds[rr * stride + w];
    } else {
        for (int rr = 0; rr < rows_here; ++rr)
            for (int w = tid; w < rd; w += NT) {
                const uint32_t v = lds[rr * stride + w];
                if (v)
                    atomicAdd(&dst[static_cast<int64_t>(rr) * rd + w], v);
            }
    }

    if (n_votes) {
        const uint32_t wsum = wave_sum(votes);
        if ((tid & 63) == 0)
            red[tid >> 6] = wsum;
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < NT / 64; ++w)
                t += red[w];
            if (t)
                atomicAdd(n_votes, t);
        }
    }
    __syncthreads();   // the LDS tile and red[] are reused by the next item
}

template <bool U16, bool D3, int RL, int RPT, int NT>
__global__ __launch_bounds__(NT) void vote_kernel(VoteKernelArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t red[NT / 64];
    __shared__ int32_t next_item;
    constexpr int ROWS = RL * RPT;
    const int tps = a.tiles_per_slice;

    if (a.items == nullptr) {
        const int tile = blockIdx.x;
        const int l = tile / tps;
        const int j0 = (tile - l * tps) * ROWS;
        const int64_t n = a.n_hits;
        const int64_t per = (n + a.split - 1) / a.split;
        const int64_t hb = static_cast<int64_t>(blockIdx.y) * per;
        const int64_t he = min(n, hb + per);
        vote_tile<U16, D3, RL, RPT, NT>(a, hb, he, l, j0, a.acc, a.split > 1, a.n_votes, lds, red);
        return;
    }
    const int32_t n_items = *a.n_items;
    int32_t it = blockIdx.x;
    for (;;) {
        if (a.work_counter) {
            if (threadIdx.x == 0)
                next_item = atomicAdd(a.work_counter, 1);
            __syncthreads();
            it = next_item;
            __syncthreads();
        }
        if (it >= n_items)
            return;
        const WorkItem w = a.items[it];
        const EventDesc ev = a.desc[w.event];
        const int l = w.tile / tps;
        const int j0 = (w.tile - l * tps) * ROWS;
        uint32_t *acc_e = a.acc + static_cast<int64_t>(w.event) * a.g.acc_dwords;
        vote_tile<U16, D3, RL, RPT, NT>(a, ev.hit_begin, ev.hit_end, l, j0, acc_e, false,
                                        a.n_votes ? a.n_votes + w.event : nullptr, lds, red);
        if (!a.work_counter)
            return;
    }
}

using VoteFn = void (*)(VoteKernelArgs);

template <bool U16, bool D3, int ROWS, int NT>
VoteFn pick_rows() {
    constexpr int RL = ROWS < 64 ? ROWS : 64;
    constexpr int RPT = ROWS / RL;
    return vote_kernel<U16, D3, RL, RPT, NT>;
}

template <bool U16, bool D3, int NT>
VoteFn pick_nt(int rows) {
    switch (rows) {
        case 4: return pick_rows<U16, D3, 4, NT>();
        case 8: return pick_rows<U16, D3, 8, NT>();
        case 16: return pick_rows<U16, D3, 16, NT>();
        case 32: return pick_rows<U16, D3, 32, NT>();
        case 64: return pick_rows<U16, D3, 64, NT>();
        case 128: return pick_rows<U16, D3, 128, NT>();
        default: return nullptr;
    }
}

template <bool U16, bool D3>
VoteFn pick_threads(int rows, int threads) {
    switch (threads) {
        case 256: return pick_nt<U16, D3, 256>(rows);
        case 512: return pick_nt<U16, D3, 512>(rows);
        case 1024: return pick_nt<U16, D3, 1024>(rows);
        default: return nullptr;
    }
}

VoteFn pick_vote(bool u16, bool d3, int rows, int threads) {
    if (u16)
        return d3 ? pick_threads<true, true>(rows, threads) : pick_threads<true, false>(rows, threads);
    return d3 ? pick_threads<false, true>(rows, threads) : pick_threads<false, false>(rows, threads);
}

__global__ void prep_kernel(EventState *state, int32_t n_events, unsigned long long *n_votes,
                            int32_t *work_counter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_events) {
        if (state) {
            state[i].key_min = 0xffffffffu;
            state[i].key_max = 0u;
            state[i].n_found = 0;
            state[i].passes = 0;
        }
        if (n_votes)
            n_votes[i] = 0ull;
    }
    if (i == 0 && work_counter)
        *work_counter = 0;
}

__global__ void prep_batch_kernel(EventState *state, int32_t max_events, const int32_t *n_events_dev,
                                  unsigned long long *n_votes, int32_t *work_counter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < max_events) {
        state[i].key_min = 0xffffffffu;
        state[i].key_max = 0u;
        state[i].n_found = 0;
        state[i].passes = 0;
        if (n_votes && i < *n_events_dev)
            n_votes[i] = 0ull;
    }
    if (i == 0 && work_counter)
        *work_counter = 0;
}

__global__ void zero_kernel(uint32_t *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0u;
}

hipError_t launch_vote(const VoteKernelArgs &a, bool u16, const VoteShape &s, dim3 grid,
                       hipStream_t stream) {
    VoteFn fn = pick_vote(u16, a.g.d0 != nullptr, s.rows, s.threads);
    if (!fn)
        return hipErrorInvalidValue;
    const size_t lds = vote_lds_bytes(s, a.g.row_dwords);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, grid, dim3(s.threads), lds, stream, a);
    return hipGetLastError();
}

}  // namespace

size_t vote_lds_bytes(const VoteShape &s, int32_t row_dwords) {
    return static_cast<size_t>(s.rows) * static_cast<size_t>(row_dwords + s.pad) * sizeof(uint32_t);
}

bool vote_shape_supported(const VoteShape &s, bool u16, int32_t row_dwords) {
    if (!pick_vote(u16, false, s.rows, s.threads))
        return false;
    if (s.pad < 0 || s.pad > 1 || s.split < 1 || s.split > 64)
        return false;
    if (s.threads / (s.rows < 64 ? s.rows : 64) < 1)
        return false;
    return vote_lds_bytes(s, row_dwords) <= 160u * 1024u - 1024u;
}

hipError_t launch_prep(EventState *state, int32_t n_events, unsigned long long *n_votes,
                       hipStream_t stream) {
    const int blocks = (n_events + 255) / 256;
    hipLaunchKernelGGL(prep_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream, state, n_events,
                       n_votes, static_cast<int32_t *>(nullptr));
    return hipGetLastError();
}

hipError_t launch_prep_batch(EventState *state, int32_t max_events, const int32_t *n_events_dev,
                             unsigned long long *n_votes, int32_t *work_counter, hipStream_t stream) {
    const int blocks = (max_events + 255) / 256;
    hipLaunchKernelGGL(prep_batch_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream, state, max_events,
                       n_events_dev, n_votes, work_counter);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t *p, int64_t n_dwords, hipStream_t stream) {
    if (n_dwords <= 0)
        return hipSuccess;
    int64_t blocks = (n_dwords + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, p, n_dwords);
    return hipGetLastError();
}

hipError_t launch_vote_single(const GridArgs &g, bool u16, const VoteShape &s, const float *x,
                              const float *y, int32_t n_hits, uint32_t *acc,
                              unsigned long long *n_votes, hipStream_t stream) {
    VoteKernelArgs a{};
    a.g = g;
    a.x = x;
    a.y = y;
    a.n_hits = n_hits;
    a.split = s.split;
    a.tiles_per_slice = (g.n_phi + s.rows - 1) / s.rows;
    a.lds_stride = g.row_dwords + s.pad;
    a.acc = acc;
    a.n_votes = n_votes;
    hipError_t e = hipSuccess;
    if (s.split > 1)
        e = launch_zero(acc, g.acc_dwords, stream);
    if (e != hipSuccess)
        return e;
    dim3 grid(static_cast<unsigned>(a.tiles_per_slice * g.n_d0), static_cast<unsigned>(s.split));
    return launch_vote(a, u16, s, grid, stream);
}

hipError_t launch_vote_batch(const GridArgs &g, bool u16, const VoteShape &s, const float *x,
                             const float *y, const EventDesc *desc, const int32_t *n_items_dev,
                             const WorkItem *items, int32_t max_items, int32_t *work_counter,
                             int32_t persistent_groups, uint32_t *acc,
                             unsigned long long *n_votes, hipStream_t stream) {
    VoteKernelArgs a{};
    a.g = g;
    a.x = x;
    a.y = y;
    a.split = 1;
    a.tiles_per_slice = (g.n_phi + s.rows - 1) / s.rows;
    a.lds_stride = g.row_dwords + s.pad;
    a.desc = desc;
    a.items = items;
    a.n_items = n_items_dev;
    a.acc = acc;
    a.n_votes = n_votes;
    unsigned blocks = static_cast<unsigned>(max_items);
    if (work_counter && persistent_groups > 0) {
        a.work_counter = work_counter;
        blocks = static_cast<unsigned>(persistent_groups < max_items ? persistent_groups : max_items);
    }
    if (blocks == 0)
        return hipSuccess;
    return launch_vote(a, u16, s, dim3(blocks), stream);
}

}  // namespace hough
