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

// 3D quotient range (every phi0 row of one hit and d0 slice): with a phi0
// table of bin centres, r in [2^-8, 2^10], d = 0 or |d| in [2^-20, 2^10] and
// |r - |d|| >= 0.03 (r + |d|):
//   den = |h - P0|^2 up to fp32 rounding (2^-21 (r + |d|)^2 absolute) lies in
//   [(r - |d|)^2, (r + |d|)^2] widened by that, i.e. within
//   [0.0009 (r + |d|)^2 (1 - 2^-10), 2^22 (1 + 2^-20)], a subset of
//   [2^-27, 2^23] and so of [2^-30, 2^30];
//   num = 2 (u - d) with |u| <= r (1 + 1e-6): |num| <= 2^12; a nonzero u - d
//   is at least 2^-45 (d = 0: u >= 2^-54 as in the 2D case; |d| >= 2^-20:
//   either |u| < |d| / 2 and |u - d| > 2^-21, or both magnitudes are at
//   least 2^-21 and the difference is a nonzero multiple of 2^-45), so every
//   nonzero numerator is in [2^-60, 2^30]; a zero numerator moves no vote.
// The test takes the fp32 r (within 3 2^-24 relative of the real one) with
// bounds pulled in by 2^-20 and the stricter 0.0301, so it implies the above.
__device__ __forceinline__ bool fast_div_3d(float r, float d, float ad) {
    const bool r_ok = r >= 0x1.00001p-8f && r <= 0x1.ffffep9f;
    const bool d_ok = d == 0.0f || (ad >= 0x1.0p-20f && ad <= 0x1.0p10f);
    return r_ok && d_ok && fabsf(r - ad) >= 0.0301f * (r + ad);
}

// Approximate bins with exact redos.  The exact fractional bin is
//   2D: kf = RN(RN(q - kappa_min) kappa_scale),     q = RN(u / h),
//   3D: kf = RN(RN(2 q - kappa_min) kappa_scale),   q = RN(num / den),
// and a vote lands in floor(kf) when 0 <= kf < n_kappa.  Both are replaced
// by kf1, an estimate of kf + E from a single FMA whose slope term P
// (q kappa_scale, or 2 q kappa_scale) is within 3 2^-24 |P| of its real value:
//   2D: kf1 = RN(u w + off),              w = RN(y kappa_scale), y the refined
//                                         reciprocal of h (a hit constant);
//   3D: kf1 = RN(RN(num rcp(den)) s2 + off), s2 = 2 kappa_scale (exact);
// with off = RN(E - kappa_min kappa_scale).  vote_near_band derives E from
// the grid so that |kf1 - (kf + E)| < E wherever |kf| <= n_kappa + 2.  Then
// kf1 in [k + 2E, k + 1) puts kf in (k, k + 1): floor(kf1) = floor(kf), and
// the range test (integer limits) decides alike; further out both miss.
// kf1 is first clamped (kf_clamp) to v in [0, n_kappa + 1/2]: a kf1 that is
// negative or at least n_kappa + 1/2 becomes n_kappa + 1/2, and kf misses
// then too (kf < kf1, or kf > kf1 - 2E > n_kappa with 2E <= 1/32).  A lane
// whose v has a fractional part below the band 2E (rounded up) redoes the
// exact kf, so every bin is the exact one; far-off lanes, whose kf1 has few
// or no fraction bits, are never flagged.
__device__ __forceinline__ float kf_offset_2d(float u, float w, float off) {
    return __builtin_fmaf(u, w, off);
}

__device__ __forceinline__ float kf_offset_3d(float num, float den, float s2, float off) {
    const float q0 = num * __builtin_amdgcn_rcpf(den);
    return __builtin_fmaf(q0, s2, off);
}

// min(kf1, n_kappa + 1/2) in bit order, given lim = bits(n_kappa + 1/2): kf1
// itself on [0, n_kappa + 1/2), else n_kappa + 1/2 (negative numbers and NaNs
// have larger bit patterns; kf1 = RN(a + off) is never -0, as off is not -0).
// Truncated to an integer it is the bin, n_kappa (the spare column) for a miss.
__device__ __forceinline__ float kf_clamp(float kf1, uint32_t lim) {
    return __uint_as_float(min(__float_as_uint(kf1), lim));
}

// v = kf_clamp(kf1) is within the band above an integer: the exact kf must decide.
__device__ __forceinline__ bool kf_in_band(float kf1, float band) {
    return __builtin_amdgcn_fractf(kf1) < band;
}

// The exact kf from the correctly rounded quotient (the division operator's
// own steps, valid in the range above).
__device__ __forceinline__ float kf_exact_2d(float u, float h, float kmin, float kscale) {
    const float q = quot_apply(u, h, quot_recip(h));
    return (q - kmin) * kscale;
}

__device__ __forceinline__ float kf_exact_3d(float num, float den, float kmin, float kscale) {
    const float q = quot_apply(num, den, quot_recip(den));
    return __builtin_fmaf(2.0f, q, -kmin) * kscale;
}

}  // namespace hough
