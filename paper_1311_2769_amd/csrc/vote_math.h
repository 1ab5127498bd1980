// fp32 quotient of the vote with the reciprocal refinement hoisted out of the
// row loop.
//
// The correctly rounded fp32 division used for the curvature (the compiler's
// default for a / b on gfx950) is Markstein's method: a reciprocal estimate
// y0 = rcp(b) is refined once with FMA (e = 1 - b y0, y = y0 + e y0), and the
// quotient is refined twice from exact FMA remainders (q0 = a y,
// r0 = a - b q0, q1 = q0 + r0 y, r1 = a - b q1, q = q1 + r1 y).  Operand
// scaling (div_scale / div_fmas) and special-value handling (div_fixup) are
// no-ops when both operands and the quotient are normal and far from the
// overflow and underflow thresholds.  Inside that range the sequence below
// performs the same operations, so its result is bit-identical to a / b;
// outside it the caller divides with the operator.
//
// In 2D the denominator is the same for all phi0 rows of a hit, so y is
// computed once per hit and each evaluation costs five FMA-pipe operations
// instead of eleven.  The 2D kernels divide u by r2/2 (both exact scalings of
// 2u and r2, so the real quotient, and with it the rounded one, is unchanged).
//
// Range of the 2D operands.  With a phi0 table of bin centres (|cos|, |sin|
// <= 1 + 1e-6, and neither closer to 0 than sin(pi / n_phi), n_phi <= 32768)
// and r2/2 in [2^-30, 2^30]: r < 2^16, so |u| <= 2^17, and a nonzero
// u = RN(RN(y c) - RN(x s)) is at least 2^-25 max(|y c|, |x s|) >= 2^-54 in
// magnitude (max(|x|, |y|) >= r / sqrt(2) >= 2^-15 and the smaller of |c|, |s|
// is at least 2^-14), so every nonzero numerator is in the range below.  A
// zero numerator may come out as +0 instead of -0, which moves no vote:
// (+-0 - kappa_min) is the same number, or +-0 when kappa_min is 0, and both
// zeros pass the range test into bin 0.
#pragma once

#include <hip/hip_runtime.h>

namespace hough {

// Denominators in [2^-30, 2^30] and numerators of magnitude in [2^-60, 2^30]
// keep every operand, remainder and quotient of the sequence normal.  (Zero
// numerators take the operator too: the FMA sequence could return +0 for -0.)
__device__ __forceinline__ bool quot_den_ok(float b) {
    return b >= 0x1.0p-30f && b <= 0x1.0p30f;
}

__device__ __forceinline__ bool quot_num_ok(float a) {
    const float m = fabsf(a);
    return m >= 0x1.0p-60f && m <= 0x1.0p30f;
}

// Refined reciprocal of b (the hoistable part).
__device__ __forceinline__ float quot_recip(float b) {
    const float y0 = __builtin_amdgcn_rcpf(b);
    const float e = __builtin_fmaf(-b, y0, 1.0f);
    return __builtin_fmaf(e, y0, y0);
}

// a / b given y = quot_recip(b), valid when quot_den_ok(b) && quot_num_ok(a).
__device__ __forceinline__ float quot_apply(float a, float b, float y) {
    const float q0 = a * y;
    const float r0 = __builtin_fmaf(-b, q0, a);
    const float q1 = __builtin_fmaf(r0, y, q0);
    const float r1 = __builtin_fmaf(-b, q1, a);
    return __builtin_fmaf(r1, y, q1);
}

// The 3D vote's fractional kappa bin from a quotient by one reciprocal:
// kf0 = (2 (num * rcp(den)) - kappa_min) * kappa_scale, with the same two
// roundings after the quotient as the exact kf.  num * rcp(den) is within
// 2^-22 |q| of the correctly rounded quotient q (rcp is within 1 ulp) when
// both operands are in the range above.
__device__ __forceinline__ float kf_one_rcp(float num, float den, float kmin, float kscale) {
    const float q0 = num * __builtin_amdgcn_rcpf(den);
    return __builtin_fmaf(2.0f, q0, -kmin) * kscale;
}

// The exact kf from the correctly rounded quotient (the division operator's
// own steps, valid in the same range).
__device__ __forceinline__ float kf_exact(float num, float den, float kmin, float kscale) {
    const float q = quot_apply(num, den, quot_recip(den));
    return __builtin_fmaf(2.0f, q, -kmin) * kscale;
}

// kf0 lies within 0.5 - near_lim of an integer: its floor may differ from
// the exact kf's, so the exact kf must decide.
__device__ __forceinline__ bool kf_near_integer(float kf0, float near_lim) {
    return fabsf(__builtin_amdgcn_fractf(kf0) - 0.5f) > near_lim;
}

}  // namespace hough
