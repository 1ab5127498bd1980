// fp32 bounds of the phi0 arcs where a hit can vote (culling only: which
// votes are cast is decided by the exact fp32 test of the vote kernels, so
// nothing here changes a result, only how many (hit, row) pairs are tried).
//
// Angles come from the device library's atan2f and asinf.  Each arc is
// widened by kArcTol radians, which is more than 100 times the error of
// either function on its whole domain; hough_selftest_angles measures that
// error against fp64 on the device.
#pragma once

#include <hip/hip_runtime.h>

namespace hough {

constexpr float kArcTol = 1e-4f;            // radians added on each side of an arc
constexpr float kArcAngleErrMax = 1e-6f;    // what hough_selftest_angles must not exceed

__device__ __forceinline__ float hit_angle(float x, float y) { return atan2f(y, x); }
__device__ __forceinline__ float arc_asin(float s) { return asinf(s); }

// Reciprocal with at most 1 ulp of error (v_rcp_f32), for normal operands.
__device__ __forceinline__ float arc_rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// q = floor(a / S) for 0 <= a < 2^16 and 1 <= S <= 2^16, given
// m = ceil(2^32 / S): a m / 2^32 exceeds a / S by less than a / 2^32 < 2^-16
// <= 1 / S, which never reaches the next integer.
__device__ __forceinline__ int div_small(int a, uint32_t m) {
    return static_cast<int>(__umulhi(static_cast<uint32_t>(a), m));
}

}  // namespace hough
