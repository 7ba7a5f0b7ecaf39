// panel_fp64.hpp -- exact potential/field integrals of one uniformly charged
// rectangle or right triangle, FP64, for gfx950 device code.
//
// Paper Sec. 2.1: the potential of a unit-density flat element is
//   Phi'(P) = integral over the element of dA / |P - s|
// and its field E'(P) = integral of (P - s)/|P - s|^3 dA; neBEM evaluates both
// in closed form for rectangles and right-angled triangles.
//
// Local frame of an element: e1 along its first edge u (length lx), e2 along
// its second edge w (length lz), e3 = e1 x e2.  The observation point is
// (X, Z, H) = ((P-o).e1, (P-o).e2, (P-o).e3).  Vertices are counter-clockwise
// about e3: rectangle (0,0) (lx,0) (lx,lz) (0,lz); right triangle (0,0)
// (lx,0) (0,lz).
//
// Closed form used here (sum over edges k with outward in-plane normal m_k,
// signed in-plane distance p_k from the projected point to the edge line):
//   Phi' = sum_k p_k Lam_k - H Omega
//   E'   = sum_k m_k Lam_k + Omega e3
// with Omega the signed solid angle the element subtends (positive for H > 0)
// and Lam_k = ln((R_b + R_a + L_k)/(R_b + R_a - L_k)) for an edge of length
// L_k between vertices at distances R_a, R_b from P, formed as
// log1p(2 L / (R_a + R_b - L)) -- accurate far from the element, where the
// argument is small -- with R_a + R_b - L assembled from two non-negative
// parts so that it stays accurate near the edge's line as well.  The solid
// angle of a triangle is the Van Oosterom-Strackee formula (IEEE Trans. Biomed. Eng. 30(2):125-126, 1983),
//   tan(Omega/2) = [R1 R2 R3] / (r1 r2 r3 + (R1.R2) r3 + (R1.R3) r2 + (R2.R3) r1)
// with R_i = P - V_i; for a planar triangle the triple product is exactly
// H * (2 * area), so no cancellation arises far away.  A rectangle is two such
// triangles sharing the diagonal; their half-angles are added through one
// atan2 of the product (D1 + iN)(D2 + iN).
//
// On the element plane (H == 0) the normal field is given its principal value
// 0 (the mean of the one-sided limits +-2 pi); Phi' is continuous there.
#pragma once
#include <hip/hip_runtime.h>

#include "fastmath_fp64.hpp"

namespace nebem {

struct Kern {
    double phi;  // Phi'
    double ex;   // E' along e1
    double ez;   // E' along e2
    double en;   // E' along e3 (= Omega)
};

constexpr double kPi = 3.14159265358979323846;

// ln((s + L)/(s - L)), s = R_a + R_b, for an edge of length L whose start
// and end points lie at along-edge coordinates lm and lp = lm + L (relative
// to the foot of the perpendicular from P to the edge's line) and distances
// Rm, Rp from P; rho2 is the squared distance from P to that line.  s - L is
// formed as (Rp - lp) + (Rm + lm), each term without cancellation
// (R - l = rho2 / (R + l) when l > 0, R + l = rho2 / (R - l) when l < 0),
// which keeps full accuracy for points close to the edge's line.
__device__ __forceinline__ double edge_log(double lm, double lp, double Rm, double Rp, double rho2, double L)
{
    const bool pp = lp > 0.0, mn = lm < 0.0;
    const double np = pp ? rho2 : Rp - lp;
    const double dp = pp ? Rp + lp : 1.0;
    const double nm = mn ? rho2 : Rm + lm;
    const double dm = mn ? Rm - lm : 1.0;
    return log1p_ratio((L + L) * dp * dm, np * dm + nm * dp);
}

// Solid-angle branch repair: the true half-angle has the sign of N and
// magnitude <= pi; atan2 of the product can land on the other side of the
// branch cut when it is near +-pi.
__device__ __forceinline__ double half_angle_fix(double half, double N)
{
    half = (N > 0.0 && half < -0.5 * kPi) ? half + 2.0 * kPi : half;
    half = (N < 0.0 && half > 0.5 * kPi) ? half - 2.0 * kPi : half;
    return half;
}

// r0sq = X^2 + Z^2 + H^2 (squared distance to the corner o), computed by the caller
__device__ __forceinline__ Kern rect_fp64(double X, double H, double Z, double lx, double lz, double r0sq)
{
    const double H2 = H * H;
    const double xm = X - lx, zm = Z - lz;
    const double X2 = X * X, Z2 = Z * Z, xm2 = xm * xm, zm2 = zm * zm;
    const double r00 = sqrt64(r0sq);
    const double r10 = sqrt64(xm2 + Z2 + H2);
    const double r11 = sqrt64(xm2 + zm2 + H2);
    const double r01 = sqrt64(X2 + zm2 + H2);
    // edges (start -> end, outward normal m, distance p of the projected point
    // from the edge line, inside positive):
    //   0 (0,0)->(lx,0)   m=(0,-1) p=Z     1 (lx,0)->(lx,lz) m=(1,0) p=lx-X
    //   2 (lx,lz)->(0,lz) m=(0,1)  p=lz-Z  3 (0,lz)->(0,0)   m=(-1,0) p=X
    const double L0 = edge_log(-X, -xm, r00, r10, Z2 + H2, lx);
    const double L1 = edge_log(-Z, -zm, r10, r11, xm2 + H2, lz);
    const double L2 = edge_log(xm, X, r11, r01, zm2 + H2, lx);
    const double L3 = edge_log(zm, Z, r01, r00, X2 + H2, lz);
    // triangles (c00,c10,c11) and (c00,c11,c01), both with [R1 R2 R3] = H lx lz
    const double N = H * lx * lz;
    const double d00_10 = X * xm + Z2 + H2;
    const double d00_11 = X * xm + Z * zm + H2;
    const double d10_11 = xm2 + Z * zm + H2;
    const double d00_01 = X2 + Z * zm + H2;
    const double d11_01 = X * xm + zm2 + H2;
    const double D1 = r00 * r10 * r11 + d00_10 * r11 + d00_11 * r10 + d10_11 * r00;
    const double D2 = r00 * r11 * r01 + d00_11 * r01 + d00_01 * r11 + d11_01 * r00;
    double half = atan2_64(N * (D1 + D2), D1 * D2 - N * N);
    half = half_angle_fix(half, N);
    const double omega = (H == 0.0) ? 0.0 : 2.0 * half;
    Kern k;
    k.phi = Z * L0 + (lx - X) * L1 + (lz - Z) * L2 + X * L3 - H * omega;
    k.ex = L1 - L3;
    k.ez = L2 - L0;
    k.en = omega;
    return k;
}

__device__ __forceinline__ Kern rtri_fp64(double X, double H, double Z, double lx, double lz, double hyp,
                                          double ihyp, double r0sq)
{
    const double H2 = H * H;
    const double xm = X - lx, zm = Z - lz;
    const double X2 = X * X, Z2 = Z * Z;
    const double r0 = sqrt64(r0sq);
    const double r1 = sqrt64(xm * xm + Z2 + H2);
    const double r2 = sqrt64(X2 + zm * zm + H2);
    // edges: 0 (0,0)->(lx,0) m=(0,-1) p=Z;  1 (lx,0)->(0,lz) m=(lz,lx)/hyp
    //        p=(lx lz - X lz - Z lx)/hyp;   2 (0,lz)->(0,0) m=(-1,0) p=X
    const double P1 = (lx * lz - X * lz - Z * lx) * ihyp;
    const double L0 = edge_log(-X, -xm, r0, r1, Z2 + H2, lx);
    const double L1 = edge_log((lx * xm - lz * Z) * ihyp, (lx * X - lz * zm) * ihyp, r1, r2, P1 * P1 + H2, hyp);
    const double L2 = edge_log(zm, Z, r2, r0, X2 + H2, lz);
    const double N = H * lx * lz;
    const double d01 = X * xm + Z2 + H2;
    const double d02 = X2 + Z * zm + H2;
    const double d12 = X * xm + Z * zm + H2;
    const double D = r0 * r1 * r2 + d01 * r2 + d02 * r1 + d12 * r0;
    const double omega = (H == 0.0) ? 0.0 : 2.0 * atan2_64(N, D);
    const double L1h = L1 * ihyp;
    Kern k;
    k.phi = Z * L0 + P1 * L1 + X * L2 - H * omega;
    k.ex = lz * L1h - L2;
    k.ez = lx * L1h - L0;
    k.en = omega;
    return k;
}

// ------------------------------------------------------------- far regime
// Same closed forms for a point whose distance R from the element's centroid
// is at least 4 element diameters D (D bounds every vertex-to-vertex and
// centroid-to-vertex distance).  Then every vertex distance r_i >= 3R/4
// >= 3D, so R_a + R_b >= 6 L for every edge: Lam_k = 2 atanh(L/(R_a + R_b))
// with an argument below 1/6, and nothing cancels.  Each triangle's solid-
// angle denominator exceeds r1 r2 r3 (1 + 3 (1 - D^2/(2 r_i r_j))) >= 1.6 R^3
// while |N| <= R D^2/2 <= R^3/32, so every arctangent argument is below 0.0194
// per triangle (0.0387 for the rectangle's sum); no octant logic, and N = 0 on
// the element's plane gives Omega = 0 by itself.  All the divisions share one
// reciprocal of the product of their denominators; its error scales every
// Lam_k and the solid angle by the same factor, which the cancellation among
// the edge terms does not amplify, so one Newton step suffices.
// The kernels select this form by the distance of the element's corner o
// (the local origin): |P - o| >= kFarDiam D implies R >= (kFarDiam - 1) D = 4 D,
// and |P - o|^2 = X^2 + Z^2 + H^2 is needed by both forms anyway.
// Beyond kVeryFarDiam D from o (R >= 24 D, every vertex >= 24 D away) the
// same evaluation runs with shorter polynomials fitted to the smaller
// ranges: atanh argument <= 1/48 (3 coefficients) and arctangent argument
// <= 2 D^2/(3.2 R^2) <= 6.5e-4 for the rectangle's sum (2 coefficients).
// Both far forms take the potential from the field components: with
// E_x' = Lam_1 - Lam_3, E_z' = Lam_2 - Lam_0 (rectangle) the edge sum
// Z Lam_0 + (lx - X) Lam_1 + (lz - Z) Lam_2 + X Lam_3 equals
// lx Lam_1 + lz Lam_2 - X E_x' - Z E_z', and for the right triangle
// Z Lam_0 + P1 Lam_1 + X Lam_2 equals lx lz Lam_1/hyp - X E_x' - Z E_z'.
// Far away each of these terms is of the size of the potential itself
// instead of lx or lz, and two products fewer are formed.
constexpr double kFarDiam = 5.0;
constexpr double kVeryFarDiam = 25.0;

template <bool VF>
struct FarPoly;
template <>
struct FarPoly<false> {
    static constexpr const double (&log)[kLogPN] = kLogP;
    static constexpr const double (&atan)[kAtanFarN] = kAtanFar;
};
template <>
struct FarPoly<true> {
    static constexpr const double (&log)[kLogPVFN] = kLogPVF;
    static constexpr const double (&atan)[kAtanVFN] = kAtanVF;
};

// Far forms: the potential is returned added to `acc` (the caller's running
// sum), which saves the caller one addition per copy.
template <bool VF>
__device__ __forceinline__ Kern rect_far(double X, double H, double Z, double lx, double lz, double r0sq, double acc)
{
    // vertex-to-point dot products and squared distances from |P - o|^2 and
    // the edges (c00 = o, c10 = o + lx e1, c11, c01 = o + lz e2); far away
    // every one of them is ~R^2 and nothing cancels
    const double d00_10 = fma(-X, lx, r0sq);
    const double d00_01 = fma(-Z, lz, r0sq);
    const double d00_11 = fma(-Z, lz, d00_10);
    const double r10sq = fma(-X, lx, d00_10 + lx * lx);
    const double r01sq = fma(-Z, lz, d00_01 + lz * lz);
    const double d10_11 = fma(-Z, lz, r10sq);
    const double d11_01 = fma(-X, lx, r01sq);
    const double r11sq = fma(-Z, lz, d10_11 + lz * lz);
    const double r00 = sqrt64_far(r0sq);
    const double r10 = sqrt64_far(r10sq);
    const double r11 = sqrt64_far(r11sq);
    const double r01 = sqrt64_far(r01sq);
    const double s0 = r00 + r10, s1 = r10 + r11, s2 = r11 + r01, s3 = r01 + r00;
    const double N2 = H * (2.0 * lx * lz);  // twice the triple product
    const double D1 = fma(fma(r00, r10, d00_10), r11, fma(d00_11, r10, d10_11 * r00));
    const double D2 = fma(fma(r00, r11, d00_11), r01, fma(d00_01, r11, d11_01 * r00));
    const double den = fma(-0.25 * N2, N2, D1 * D2);
    // one reciprocal for 1/s0 .. 1/s3 and 1/den
    const double a = s0 * s1, b = s2 * s3, ab = a * b;
    const double inv = rcp64_common(ab * den);
    const double iden = ab * inv, iab = den * inv;
    const double ia = iab * b, ib = iab * a;
    const double L0 = two_atanh_poly(lx * (ia * s1), FarPoly<VF>::log);
    const double L1 = two_atanh_poly(lz * (ia * s0), FarPoly<VF>::log);
    const double L2 = two_atanh_poly(lx * (ib * s3), FarPoly<VF>::log);
    const double L3 = two_atanh_poly(lz * (ib * s2), FarPoly<VF>::log);
    const double omega = two_atan_half(N2 * (D1 + D2) * iden, FarPoly<VF>::atan);
    Kern k;
    k.ex = L1 - L3;
    k.ez = L2 - L0;
    k.phi = fma(-Z, k.ez, fma(-X, k.ex, fma(lz, L2, fma(lx, L1, fma(-H, omega, acc)))));
    k.en = omega;
    return k;
}

template <bool VF>
__device__ __forceinline__ Kern rtri_far(double X, double H, double Z, double lx, double lz, double hyp,
                                         double r0sq, double acc)
{
    // dot products (P - v_a).(P - v_b) and squared distances from |P - o|^2
    // (v_0 = o, v_1 = o + lx e1, v_2 = o + lz e2, e1 . e2 = 0)
    const double d01 = fma(-X, lx, r0sq);
    const double d02 = fma(-Z, lz, r0sq);
    const double d12 = fma(-Z, lz, d01);
    const double r0 = sqrt64_far(r0sq);
    const double r1 = sqrt64_far(fma(-X, lx, d01 + lx * lx));
    const double r2 = sqrt64_far(fma(-Z, lz, d02 + lz * lz));
    const double s0 = r0 + r1, s1 = r1 + r2, s2 = r2 + r0;
    const double lxlz = lx * lz;
    const double N2 = H * (2.0 * lxlz);  // twice the triple product
    const double D = fma(fma(r0, r1, d01), r2, fma(d02, r1, d12 * r0));
    // one reciprocal for 1/s0, 1/s1, 1/s2 and 1/D
    const double a = s0 * s1, b = a * s2;
    const double inv = rcp64_common(b * D);
    const double iD = b * inv, ib = D * inv;
    const double ia = ib * s2;
    const double L0 = two_atanh_poly(lx * (ia * s1), FarPoly<VF>::log);
    const double L1h = two_atanh_over(ia * s0, hyp, FarPoly<VF>::log);  // Lam_1 / hyp
    const double L2 = two_atanh_poly(lz * (ib * a), FarPoly<VF>::log);
    const double omega = two_atan_half(N2 * iD, FarPoly<VF>::atan);
    Kern k;
    k.ex = fma(lz, L1h, -L2);
    k.ez = fma(lx, L1h, -L0);
    k.phi = fma(-Z, k.ez, fma(-X, k.ex, fma(lxlz, L1h, fma(-H, omega, acc))));
    k.en = omega;
    return k;
}

// Two right triangles that share their right-angle corner o and one leg:
// triangle 1 with legs a along e1 and c along e2 (vertices o, A = o + a e1,
// C = o + c e2) and triangle 2 with legs c along e2 and b along -e1
// (vertices o, C, B = o - b e1), both with normal e3 -- the two halves of a
// triangle cut at the foot of its altitude.  Triangle 2 in its own frame
// (e2, -e1, e3) sees the point at (Z, H, -X), and its closed form is
// rtri_far's with lx = c, lz = b; evaluated together, the two share the
// distances to o and C, the edge o-C with its logarithm, and one reciprocal
// for all seven divisions (its error scales every quotient of both by the
// same factor).  Four square roots and five edge logarithms per pair instead
// of six and six.  k2 is in triangle 2's frame; the potentials are returned
// added to acc1, acc2.
template <bool VF>
__device__ __forceinline__ void rtri_pair_far(double X, double H, double Z, double a, double b, double c,
                                              double hyp1, double hyp2, double r0sq, double acc1, double acc2,
                                              Kern &k1, Kern &k2)
{
    const double d0A = fma(-X, a, r0sq);  // (P - o).(P - A)
    const double d0C = fma(-Z, c, r0sq);  // (P - o).(P - C)
    const double dAC = fma(-Z, c, d0A);   // (P - A).(P - C)
    const double d0B = fma(X, b, r0sq);   // (P - o).(P - B)
    const double dCB = fma(X, b, d0C);    // (P - C).(P - B)
    const double r0 = sqrt64_far(r0sq);
    const double rA = sqrt64_far(fma(-X, a, d0A + a * a));
    const double rC = sqrt64_far(fma(-Z, c, d0C + c * c));
    const double rB = sqrt64_far(fma(X, b, d0B + b * b));
    const double s0A = r0 + rA, sAC = rA + rC, sC0 = rC + r0, sCB = rC + rB, sB0 = rB + r0;
    const double D1 = fma(fma(r0, rA, d0A), rC, fma(d0C, rA, dAC * r0));
    const double D2 = fma(fma(r0, rC, d0C), rB, fma(d0B, rC, dCB * r0));
    // one reciprocal for 1/s (five edges) and 1/D1, 1/D2
    const double a1 = s0A * sAC, b1 = a1 * sC0, P1 = b1 * D1;
    const double a2 = sCB * sB0, P2 = a2 * D2;
    const double inv = rcp64_common(P1 * P2);
    const double i1 = P2 * inv, i2 = P1 * inv;  // 1/P1, 1/P2
    const double iD1 = b1 * i1, ib1 = D1 * i1, ia1 = ib1 * sC0;
    const double iD2 = a2 * i2, ia2 = D2 * i2;
    const double L0A = two_atanh_poly(a * (ia1 * sAC), FarPoly<VF>::log);
    const double LACh = two_atanh_over(ia1 * s0A, hyp1, FarPoly<VF>::log);  // Lam_AC / hyp1
    const double LC0 = two_atanh_poly(c * (ib1 * a1), FarPoly<VF>::log);     // the shared edge
    const double LCBh = two_atanh_over(ia2 * sB0, hyp2, FarPoly<VF>::log);  // Lam_CB / hyp2
    const double LB0 = two_atanh_poly(b * (ia2 * sCB), FarPoly<VF>::log);
    const double om1 = two_atan_half(H * (2.0 * a * c) * iD1, FarPoly<VF>::atan);
    const double om2 = two_atan_half(H * (2.0 * c * b) * iD2, FarPoly<VF>::atan);
    k1.ex = fma(c, LACh, -LC0);
    k1.ez = fma(a, LACh, -L0A);
    k1.phi = fma(-Z, k1.ez, fma(-X, k1.ex, fma(a * c, LACh, fma(-H, om1, acc1))));
    k1.en = om1;
    // triangle 2: frame coordinates (Z, -X), legs c (along its e1) and b
    k2.ex = fma(b, LCBh, -LB0);
    k2.ez = fma(c, LCBh, -LC0);
    k2.phi = fma(X, k2.ez, fma(-Z, k2.ex, fma(c * b, LCBh, fma(-H, om2, acc2))));
    k2.en = om2;
}

}  // namespace nebem
