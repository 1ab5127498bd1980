// Device self-tests.
//  - The vote's division fast path (vote_math.h): over n pseudo-random operand
//    pairs drawn across the whole range where the fast path is used, the
//    hoisted-reciprocal sequence must equal the division operator bit for bit.
//  - The angle functions of the culling arcs (arc_math.h): their largest
//    absolute error against fp64 over n pseudo-random arguments from their
//    whole domain in hit_prep_kernel.
//  - The approximate bins (vote_math.h), 3D and 2D: wherever kf1 is outside
//    the band above an integer, its bin (or its miss) must be the exact kf's.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "hough.h"
#include "vote_math.h"
#include "arc_math.h"
#include "hough_impl.h"

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea and Flood, 2014).
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// A float with a random mantissa (sometimes all ones or zero) and an
// exponent uniform in [lo, hi].
__device__ __forceinline__ float draw(uint64_t bits, int lo, int hi) {
    uint32_t mant = static_cast<uint32_t>(bits) & 0x7fffffu;
    const uint32_t kind = static_cast<uint32_t>(bits >> 23) & 15u;
    if (kind == 0)
        mant = 0x7fffffu;
    else if (kind == 1)
        mant = 0u;
    else if (kind == 2)
        mant &= 0x7f0000u;
    const int e = lo + static_cast<int>((bits >> 32) % static_cast<uint64_t>(hi - lo + 1));
    const uint32_t sign = static_cast<uint32_t>(bits >> 63) << 31;
    return __uint_as_float(sign | (static_cast<uint32_t>(e + 127) << 23) | mant);
}

__global__ void divide_check_kernel(int64_t n, uint64_t seed, unsigned long long *bad, unsigned long long *used) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long nbad = 0, nused = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t h1 = mix64(seed + 2 * static_cast<uint64_t>(i));
        const uint64_t h2 = mix64(seed + 2 * static_cast<uint64_t>(i) + 1);
        const float b = fabsf(draw(h1, -31, 31));     // denominators are positive squares
        const float a = draw(h2, -62, 32);
        if (!hough::quot_den_ok(b) || !hough::quot_num_ok(a))
            continue;
        ++nused;
        const float fast = hough::quot_apply(a, b, hough::quot_recip(b));
        const float ref = a / b;
        if (__float_as_uint(fast) != __float_as_uint(ref))
            ++nbad;
    }
    if (nbad)
        atomicAdd(bad, nbad);
    if (nused)
        atomicAdd(used, nused);
}


__device__ __forceinline__ void max_err(unsigned *slot, double err) {
    // non-negative floats order like their bit patterns
    const float e = static_cast<float>(err);
    atomicMax(slot, __float_as_uint(e != e ? INFINITY : e));
}

__global__ void angle_check_kernel(int64_t n, uint64_t seed, unsigned *worst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    double e_atan = 0.0, e_asin = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t h1 = mix64(seed + 3 * static_cast<uint64_t>(i));
        const uint64_t h2 = mix64(seed + 3 * static_cast<uint64_t>(i) + 1);
        const uint64_t h3 = mix64(seed + 3 * static_cast<uint64_t>(i) + 2);
        // hit coordinates: r in [2^-30, 2^30], either coordinate may be 0
        float x = draw(h1, -31, 29);
        float y = draw(h2, -31, 29);
        const uint32_t k = static_cast<uint32_t>(h3) & 63u;
        if (k == 0)
            x = 0.0f;
        else if (k == 1)
            y = 0.0f;
        else if (k < 8)
            y = x * (1.0f + static_cast<float>(k) * 1e-7f);   // near the diagonals
        const double ref_a = atan2(static_cast<double>(y), static_cast<double>(x));
        e_atan = fmax(e_atan, fabs(static_cast<double>(hough::hit_angle(x, y)) - ref_a));
        // sine bounds: uniform in [-1, 1], or within 2^-k of +-1
        float s = static_cast<float>(static_cast<int64_t>(h3 >> 40) - (1ll << 23)) * 0x1.0p-23f;
        if (((h3 >> 8) & 3u) == 0)
            s = copysignf(1.0f - ldexpf(1.0f, -static_cast<int>((h3 >> 10) % 25u)), s);
        s = fminf(fmaxf(s, -1.0f), 1.0f);
        e_asin = fmax(e_asin, fabs(static_cast<double>(hough::arc_asin(s)) - asin(static_cast<double>(s))));
    }
    max_err(worst, e_atan);
    max_err(worst + 1, e_asin);
}


__device__ __forceinline__ int canonical_bin(float kf, int nk) {
    return (kf >= 0.0f && kf < static_cast<float>(nk)) ? static_cast<int>(kf) : -1;
}

// Operands of the fast paths, with the exact kf placed across the kappa band
// (half of the draws within a few E of an integer, a tenth outside the
// band).  form 0: 3D, den in [2^-27, 2^23]; form 1: 2D, h = r2/2 in
// [2^-30, 2^30], an eighth of them h = 1 (the straight-line records).
__global__ void near_check_kernel(int64_t n, uint64_t seed, int form, float kmin, float kscale, int nk,
                                  float band, float off, unsigned long long *bad, unsigned long long *redone,
                                  unsigned long long *used) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const float E = 0.5f * band;
    unsigned long long nbad = 0, nredo = 0, nused = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t h1 = mix64(seed + 2 * static_cast<uint64_t>(i));
        const uint64_t h2 = mix64(seed + 2 * static_cast<uint64_t>(i) + 1);
        float den = form == 0 ? fabsf(draw(h1, -27, 22)) : fabsf(draw(h1, -30, 29));
        if (form == 1 && ((h1 >> 60) & 7u) == 0u)
            den = 1.0f;
        const float u01 = static_cast<float>(h2 >> 40) * 0x1.0p-24f;
        const uint32_t kind = static_cast<uint32_t>(h2) & 15u;
        float kf_t;
        if (kind < 2) {
            kf_t = (kind ? static_cast<float>(nk) + 2.0f : -102.0f) + 100.0f * u01;   // outside the band
        } else if (kind < 9) {
            const float m = floorf(u01 * static_cast<float>(nk + 3)) - 1.0f;            // an integer of the band
            const float dev = (static_cast<float>((h2 >> 8) & 0xffffu) * 0x1.0p-16f - 0.5f) * 8.0f * E;
            kf_t = m + dev;
        } else {
            kf_t = -2.0f + u01 * static_cast<float>(nk + 4);
        }
        const float q_t = form == 0 ? 0.5f * (kf_t / kscale + kmin) : kf_t / kscale + kmin;
        const float num = q_t * den;
        if (!hough::quot_den_ok(den) || !hough::quot_num_ok(num))
            continue;
        ++nused;
        float kf1, kf;
        if (form == 0) {
            kf1 = hough::kf_offset_3d(num, den, 2.0f * kscale, off);
            kf = hough::kf_exact_3d(num, den, kmin, kscale);
        } else {
            kf1 = hough::kf_offset_2d(num, hough::quot_recip(den) * kscale, off);
            kf = hough::kf_exact_2d(num, den, kmin, kscale);
        }
        // the vote's bin: the clamped value truncated, n_kappa for a miss
        const float v = hough::kf_clamp(kf1, __float_as_uint(static_cast<float>(nk) + 0.5f));
        const int b1 = static_cast<int>(v);
        if (hough::kf_in_band(v, band))
            ++nredo;
        else if ((b1 < nk ? b1 : -1) != canonical_bin(kf, nk))
            ++nbad;
    }
    if (nbad)
        atomicAdd(bad, nbad);
    if (nredo)
        atomicAdd(redone, nredo);
    if (nused)
        atomicAdd(used, nused);
}

}  // namespace

extern "C" hough_status hough_selftest_divide(int64_t n, uint64_t seed, uint64_t *mismatches, uint64_t *checked) {
    if (n < 0 || !mismatches)
        return HOUGH_EINVAL;
    unsigned long long *d = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d), 2 * sizeof(unsigned long long)) != hipSuccess)
        return HOUGH_ENOMEM;
    hough_status st = HOUGH_OK;
    unsigned long long h[2] = {0, 0};
    if (hipMemset(d, 0, 2 * sizeof(unsigned long long)) != hipSuccess)
        st = HOUGH_EDEVICE;
    if (st == HOUGH_OK) {
        hipLaunchKernelGGL(divide_check_kernel, dim3(4096), dim3(256), 0, 0, n, seed, d, d + 1);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
            st = HOUGH_EDEVICE;
    }
    (void)hipFree(d);
    *mismatches = h[0];
    if (checked)
        *checked = h[1];
    return st;
}

extern "C" hough_status hough_selftest_angles(int64_t n, uint64_t seed, float *max_err_atan2, float *max_err_asin) {
    if (n < 0 || !max_err_atan2 || !max_err_asin)
        return HOUGH_EINVAL;
    unsigned *d = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d), 2 * sizeof(unsigned)) != hipSuccess)
        return HOUGH_ENOMEM;
    hough_status st = HOUGH_OK;
    unsigned h[2] = {0u, 0u};
    if (hipMemset(d, 0, 2 * sizeof(unsigned)) != hipSuccess)
        st = HOUGH_EDEVICE;
    if (st == HOUGH_OK) {
        hipLaunchKernelGGL(angle_check_kernel, dim3(2048), dim3(256), 0, 0, n, seed, d);
        if (hipGetLastError() != hipSuccess || hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
            st = HOUGH_EDEVICE;
    }
    (void)hipFree(d);
    float a, b;
    memcpy(&a, &h[0], sizeof a);
    memcpy(&b, &h[1], sizeof b);
    *max_err_atan2 = a;
    *max_err_asin = b;
    return st;
}

extern "C" hough_status hough_selftest_near(int64_t n, uint64_t seed, float kappa_min, float kappa_scale,
                                            int32_t n_kappa, int32_t form, uint64_t *mismatches, uint64_t *redone,
                                            uint64_t *checked) {
    if (n < 0 || n_kappa < 1 || (form != 0 && form != 1) || !mismatches || !redone || !checked)
        return HOUGH_EINVAL;
    hough::GridArgs g{};
    g.kappa_min = kappa_min;
    g.kappa_scale = kappa_scale;
    g.n_kappa = n_kappa;
    float band = 0.0f, off = 0.0f;
    if (!hough::vote_near_band(g, &band, &off))
        return HOUGH_EINVAL;     // the grid never takes approximate bins
    unsigned long long *d = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d), 3 * sizeof(unsigned long long)) != hipSuccess)
        return HOUGH_ENOMEM;
    hough_status st = HOUGH_OK;
    unsigned long long h[3] = {0, 0, 0};
    if (hipMemset(d, 0, sizeof h) != hipSuccess)
        st = HOUGH_EDEVICE;
    if (st == HOUGH_OK) {
        hipLaunchKernelGGL(near_check_kernel, dim3(4096), dim3(256), 0, 0, n, seed, static_cast<int>(form), kappa_min,
                           kappa_scale, n_kappa, band, off, d, d + 1, d + 2);
        if (hipGetLastError() != hipSuccess || hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
            st = HOUGH_EDEVICE;
    }
    (void)hipFree(d);
    *mismatches = h[0];
    *redone = h[1];
    *checked = h[2];
    return st;
}
