// fastmath_fp64.hpp -- FP64 reciprocal, square root, logarithm of 1 + a ratio
// and two-argument arctangent for the element kernels.
//
// Arguments here are finite and of normal magnitude (lengths of metres down
// to nanometres, squared), so the special-value and subnormal handling of the
// general library routines is left out.  Accuracy: rcp64 / div64 / sqrt64
// about 1 ulp; log1p_ratio and atan2_64 a few ulp (polynomial truncation
// < 5e-18, see gen_poly.py; the rest is FP64 rounding).
#pragma once
#include <hip/hip_runtime.h>

#include "poly_coeffs.hpp"

namespace nebem {

constexpr double kPiD = 3.141592653589793;
constexpr double kPi2D = 1.5707963267948966;
constexpr double kPi4D = 0.7853981633974483;
constexpr double kSqrtHalf = 0.7071067811865476;
constexpr double kTanPi8 = 0.41421356237309503;  // sqrt2 - 1

// 1/d: hardware estimate, two Newton steps (quadratic convergence)
__device__ __forceinline__ double rcp64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// 1/d from the hardware estimate with one Newton step (the estimate is good
// to ~5e-8 relative on gfx950, the result to ~2e-15): for a reciprocal whose
// error scales a whole set of quotients by one common factor
__device__ __forceinline__ double rcp64_common(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}

// n/d with a final residual correction
__device__ __forceinline__ double div64(double n, double d)
{
    const double r = rcp64(d);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

// sqrt(x) for x > 0 (no zero test).  With y = rsq(x) = (1 + e)/sqrt(x):
// g = x y refined once has error ~1.5 e^2; the final residual correction
// (x - g^2) h then needs h = y/2 only to relative accuracy e (its error
// multiplies a correction of size e^2), leaving ~1.5 e^3 plus rounding.
__device__ __forceinline__ double sqrt64_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    const double h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    return fma(fma(-g, g, x), h, g);
}

// sqrt(x) for x > 0 with one Newton step on the estimate g = x rsq(x):
// g + (x - g^2) y/2 = sqrt(x) (1 - 1.5 e^2 + O(e^3)) with e the estimate's
// relative error (~5e-8 on gfx950): ~4e-15 relative, two operations fewer
// than sqrt64_pos.  For the far-regime forms, where every distance enters
// through sums r_a + r_b whose relative error passes unamplified into the
// edge logarithms, and the per-element error is set by the cancellation
// among edge terms (~R/D ulps) rather than by the distances.
__device__ __forceinline__ double sqrt64_far(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y;
    return fma(fma(-g, g, x), 0.5 * y, g);
}

// sqrt(x), x >= 0 (0 for x == 0, where the estimate is infinite)
__device__ __forceinline__ double sqrt64(double x) { return x > 0.0 ? sqrt64_pos(x) : 0.0; }

template <int N>
__device__ __forceinline__ double horner(const double (&c)[N], double z)
{
    double acc = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) acc = fma(acc, z, c[k]);
    return acc;
}

// ln(1 + nn/dd) for nn >= 0, dd > 0, with one division:
//   nn/dd < sqrt2 - 1:  s = nn/(nn + 2 dd), result 2 atanh(s);
//   otherwise           dd + nn = m1 2^e1, dd = m2 2^e2 (m in [1/2, 1)), the
//                       ratio m1/m2 brought into [sqrt(1/2), sqrt2) with e,
//                       s = (m1 - m2)/(m1 + m2), result e ln2 + 2 atanh(s);
// in both cases |s| <= (sqrt2 - 1)/(sqrt2 + 1) and 2 atanh(s) = 2s + s z P(z).
__device__ __forceinline__ double log1p_ratio(double nn, double dd)
{
    const double x = dd + nn;
    double m1 = __builtin_amdgcn_frexp_mant(x), m2 = __builtin_amdgcn_frexp_mant(dd);
    int e = __builtin_amdgcn_frexp_exp(x) - __builtin_amdgcn_frexp_exp(dd);
    const bool lo = m1 < kSqrtHalf * m2, hi = m1 >= (2.0 * kSqrtHalf) * m2;
    m1 = lo ? m1 + m1 : m1;
    m2 = hi ? m2 + m2 : m2;
    e += hi ? 1 : 0;
    e -= lo ? 1 : 0;
    const bool small = nn < kTanPi8 * dd;
    const double num = small ? nn : m1 - m2;
    const double den = small ? fma(2.0, dd, nn) : m1 + m2;
    const double ee = small ? 0.0 : (double)e;
    const double s = div64(num, den);
    const double z = s * s;
    const double t = fma(s * z, horner(kLogP, z), s + s);
    return fma(ee, kLn2Hi, fma(ee, kLn2Lo, t));
}

// 2 atanh(t) = t (2 + z P(z)) and atan(t) = t + t z Q(z), z = t^2, with the
// coefficient set fitted to the range t is known to lie in (kLogP: t up to
// (sqrt2 - 1)/(sqrt2 + 1); kLogPVF: 1/48; kAtanFar: 0.039; kAtanVF: 6.5e-4)
template <int N>
__device__ __forceinline__ double two_atanh_poly(double t, const double (&c)[N])
{
    const double z = t * t;
    return t * fma(z, horner(c, z), 2.0);  // t (2 + z P(z)), about one ulp
}

// 2 atanh(L u) / L, for a caller that needs the logarithm divided by L
template <int N>
__device__ __forceinline__ double two_atanh_over(double u, double L, const double (&c)[N])
{
    const double t = L * u;
    const double z = t * t;
    return u * fma(z, horner(c, z), 2.0);
}

// 2 atan(u/2) from u: 2 atan(t) = u + u w Q(w/4)/4 with w = u^2; the
// coefficients of Q are rescaled by powers of 4 (exact) at compile time
template <int N>
__device__ __forceinline__ double two_atan_half(double u, const double (&c)[N])
{
    const double w = u * u;
    double acc = c[N - 1];
    double sc = 1.0;
#pragma unroll
    for (int k = 0; k < N; ++k) sc *= 0.25;
    acc *= sc;
#pragma unroll
    for (int k = N - 2; k >= 0; --k) {
        sc *= 4.0;
        acc = fma(acc, w, c[k] * sc);
    }
    return fma(u * w, acc, u);
}

// atan2(y, x) with one division: t = min/max of |x|, |y| reduced to
// [0, tan(pi/8)] (past it via (min - max)/(min + max) and + pi/4), then
// atan(s) = s + s z Q(z); octant and sign restored.  atan2(+-0, x < 0) = +-pi.
__device__ __forceinline__ double atan2_64(double y, double x)
{
    const double ay = fabs(y), ax = fabs(x);
    const double mx = fmax(ax, ay), mn = fmin(ax, ay);
    const bool red = mn > kTanPi8 * mx;
    const double num = red ? mn - mx : mn;
    const double den = red ? mn + mx : mx;
    const double s = div64(num, den);
    const double z = s * s;
    double a = fma(s * z, horner(kAtanQ, z), s);
    a = red ? a + kPi4D : a;
    a = ay > ax ? kPi2D - a : a;
    a = x < 0.0 ? kPiD - a : a;
    a = mx > 0.0 ? a : 0.0;
    return copysign(a, y);
}

}  // namespace nebem
