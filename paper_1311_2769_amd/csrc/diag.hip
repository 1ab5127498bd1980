// Throughput probes used to price the vote kernel against its roofs: the
// conflict-free, no-return 32-bit LDS atomic add (the vote's one memory
// operation) and the plain fp32 VALU operation (unpacked, unfused: the vote's
// arithmetic), each saturating every compute unit.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hough.h"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kLdsWords = 4096;
constexpr int kBlocksPerCu = 8;

__global__ __launch_bounds__(kProbeThreads) void lds_add_probe(int iters, unsigned long long *out) {
    __shared__ uint32_t buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kProbeThreads)
        buf[i] = 0u;
    __syncthreads();
    // Each instruction of a wavefront adds to 64 consecutive dwords: one per bank.
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            __hip_atomic_fetch_add(&buf[(k * kProbeThreads + threadIdx.x) & (kLdsWords - 1)], 1u,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < kLdsWords; i += kProbeThreads)
        s += buf[i];
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0)
        atomicAdd(out, s);
}

__global__ __launch_bounds__(kProbeThreads) void valu_probe(int iters, float m, float c, float *out) {
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        a[k] = 1.0f + 1e-3f * static_cast<float>(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = a[k] * m;
            a[k] = a[k] - c;
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        s += a[k];
    if (s == 12345.0f)   // never true for these inputs; keeps the chains live
        out[0] = s;
}

template <typename Launch>
hipError_t time_launch(Launch launch, float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        launch();                                     // warm-up
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    if (e == hipSuccess)
        e = hipEventElapsedTime(ms, e0, e1);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

extern "C" hough_status hough_diag_rates(double *lds_atomics_per_s, double *valu_ops_per_s) {
    if (!lds_atomics_per_s || !valu_ops_per_s)
        return HOUGH_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return HOUGH_EDEVICE;
    const int blocks = (prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256) * kBlocksPerCu;
    void *buf = nullptr;
    if (hipMalloc(&buf, 64) != hipSuccess)
        return HOUGH_ENOMEM;
    hough_status st = HOUGH_OK;
    if (hipMemset(buf, 0, 64) != hipSuccess)
        st = HOUGH_EDEVICE;
    const int lds_iters = 2048;
    const int valu_iters = 8192;
    float ms_lds = 0.0f, ms_valu = 0.0f;
    if (st == HOUGH_OK &&
        time_launch([&] {
            hipLaunchKernelGGL(lds_add_probe, dim3(blocks), dim3(kProbeThreads), 0, nullptr, lds_iters,
                               static_cast<unsigned long long *>(buf));
        }, &ms_lds) != hipSuccess)
        st = HOUGH_EDEVICE;
    if (st == HOUGH_OK &&
        time_launch([&] {
            hipLaunchKernelGGL(valu_probe, dim3(blocks), dim3(kProbeThreads), 0, nullptr, valu_iters, 1.0000001f,
                               1e-7f, static_cast<float *>(buf));
        }, &ms_valu) != hipSuccess)
        st = HOUGH_EDEVICE;
    (void)hipFree(buf);
    if (st != HOUGH_OK || ms_lds <= 0.0f || ms_valu <= 0.0f)
        return st == HOUGH_OK ? HOUGH_EDEVICE : st;
    const double threads = static_cast<double>(blocks) * kProbeThreads;
    *lds_atomics_per_s = threads * lds_iters * 16.0 / (ms_lds * 1e-3);
    *valu_ops_per_s = threads * valu_iters * 16.0 / (ms_valu * 1e-3);
    return HOUGH_OK;
}
