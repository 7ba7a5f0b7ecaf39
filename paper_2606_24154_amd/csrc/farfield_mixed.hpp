// farfield_mixed.hpp -- far-field potential/field of one element copy for the
// mixed-precision path: FP64 monopole plus an FP32 quadrature correction.
//
// Far from an element (R = distance to its centroid, D = its diameter, R
// many D) the integrand of Sec. 2.1 is smooth, and a quadrature
// rule with nodes s_k = c + delta_k and weights w_k (sum 1) gives
//   Phi' = A sum_k w_k / R_k,   E' = A sum_k w_k (p - delta_k) / R_k^3
// with p = P - c, R_k = |p - delta_k|.  The centroid term A/R_c is evaluated
// in FP64; the remainder is carried in FP32 in difference form so that no
// cancellation happens against the monopole:
//   1/R_k - 1/R_c = t_k / (R_k R_c),  t_k = R_c - R_k = (2 p.delta_k - |delta_k|^2)/(R_c + R_k)
//   1/R_k^3 - 1/R_c^3 = t_k / (R_k R_c) (1/R_k^2 + 1/(R_k R_c) + 1/R_c^2).
// Its FP32 rounding is then relative to the correction, itself O((D/R)^2)
// of the monopole.
//
// Tiers (per-element truncation error of E against the exact integral,
// measured; it falls as a power of D/R):
//   rectangle      24 D <= R < 32 D: 2 x 2 Gauss-Legendre (<= 8e-8)
//   right triangle 48 D <= R < 96 D: the 3-point interior degree-2 rule
//                  (<= 7e-8; A. H. Stroud, Approximate Calculation of
//                  Multiple Integrals, 1971)
// Beyond (rectangle R >= 32 D, triangle R >= 96 D) the correction is the
// quadrupole term of the multipole expansion about the centroid instead of a
// quadrature: with the element's second central moments M (per unit area, in
// its plane; rectangle diag(lx^2, lz^2)/12, right triangle lx^2/18, lz^2/18,
// off-diagonal -lx lz/36), q = p.M p and t = tr M,
//   Phi' = A/R + A (3q - R^2 t)/(2 R^5)
//   E'   = A p/R^3 + A/R^5 [(5 (3q - R^2 t)/(2 R^2) + t) p - 3 M p].
// Its truncation error there (E: <= 5e-8 rectangle, <= 3.5e-8 triangle) is
// below the 3-point rule's at 48 D.  Nearer copies are evaluated with the
// exact closed forms (a 3 x 3 or 7-point rule there costs as much as the
// exact far-regime form and contributed most of the error of sums).
#pragma once
#include <hip/hip_runtime.h>

#include "panel_fp64.hpp"

namespace nebem {

// Gauss-Legendre nodes/weights on [0, 1]
struct GL2 {
    static constexpr int n = 2;
    static constexpr float x[2] = {0.21132486540518711775f, 0.78867513459481288225f};
    static constexpr float w[2] = {0.5f, 0.5f};
};

// triangle rule in (s, t) on s, t >= 0, s + t <= 1 (area coordinates of the
// vertices o + u and o + w); weights sum to 1
struct TriR3 {
    static constexpr int n = 3;
    static constexpr float s[3] = {0.66666666666666666667f, 0.16666666666666666667f, 0.16666666666666666667f};
    static constexpr float t[3] = {0.16666666666666666667f, 0.66666666666666666667f, 0.16666666666666666667f};
    static constexpr float w[3] = {0.33333333333333333333f, 0.33333333333333333333f, 0.33333333333333333333f};
};

// FP32 correction accumulators over the nodes of one rule
struct FarAcc {
    float cphi;  // sum w t/R_k                         (x A/R_c  -> potential correction)
    float gp;    // sum w t/R_k (1/R_k^2 + 1/(R_k R_c) + 1/R_c^2)   (x A p/R_c)
    float gx, gz;  // sum w delta/R_k^3                 (x -A)
};

__device__ __forceinline__ void far_node(float px, float pz, float rc2, float rc, float ic, float ic2, float dx,
                                         float dz, float w, FarAcc &a)
{
    const float d = fmaf(px, dx, pz * dz);
    const float num = fmaf(2.0f, d, -fmaf(dx, dx, dz * dz));  // 2 p.delta - |delta|^2
    const float rk2 = rc2 - num;
    const float ik = __builtin_amdgcn_rsqf(rk2);
    const float rk = rk2 * ik;
    const float t = num * __builtin_amdgcn_rcpf(rc + rk);  // R_c - R_k
    const float wq = w * (t * ik);
    a.cphi += wq;
    a.gp = fmaf(wq, fmaf(ik, ik + ic, ic2), a.gp);
    const float w3 = w * (ik * ik * ik);
    a.gx = fmaf(w3, dx, a.gx);
    a.gz = fmaf(w3, dz, a.gz);
}

// Corrections per unit area, summed in FP32 over the copies of one element
// and added to the FP64 sums once, scaled by the area.  Each is at most a few
// 1e-3 of its copy's monopole, so the FP32 sum over ~100 copies keeps them
// to ~1e-8 of the element's field, below the tiers' truncation error.
struct FarCorr {
    float p, x, z, n;
};

// FP64 monopole A/R_c, A p/R_c^3 of one copy added to (sp, sx, sz, sn).
// 1/R_c from the FP32 estimate fic (relative error <= 2^-23) by one Newton
// step (error ~1.5 x 2^-46), far inside the mixed path's error budget.
__device__ __forceinline__ void monopole_fp64(double px, double pz, double ph, double rc2, float fic, double area,
                                              double &sp, double &sx, double &sz, double &sn)
{
    double ir = (double)fic;
    ir = ir * (1.5 - 0.5 * rc2 * ir * ir);
    const double air = area * ir;
    const double air3 = air * ir * ir;
    sp += air;
    sx = fma(air3, px, sx);
    sz = fma(air3, pz, sz);
    sn = fma(air3, ph, sn);
}

// p = (px, pz, ph): point relative to the element centroid in the element
// frame (FP64); rc2 = |p|^2.  Adds the monopole of Phi', E' (local frame) to
// (sp, sx, sz, sn) and the quadrature correction per unit area to c.
template <int KIND>
__device__ __forceinline__ void far_mixed(double px, double pz, double ph, double rc2, double lx, double lz,
                                          double area, double &sp, double &sx, double &sz, double &sn, FarCorr &c)
{
    const float fx = (float)px, fz = (float)pz;
    const float frc2 = (float)rc2;
    const float fic = __builtin_amdgcn_rsqf(frc2);
    const float frc = frc2 * fic;
    const float fic2 = fic * fic;
    const float flx = (float)lx, flz = (float)lz;
    FarAcc a = {0.0f, 0.0f, 0.0f, 0.0f};
    if (KIND == 0) {
#pragma unroll
        for (int i = 0; i < GL2::n; ++i)
#pragma unroll
            for (int j = 0; j < GL2::n; ++j)
                far_node(fx, fz, frc2, frc, fic, fic2, flx * (GL2::x[i] - 0.5f), flz * (GL2::x[j] - 0.5f),
                         GL2::w[i] * GL2::w[j], a);
    } else {
        const float third = 0.33333333333333333333f;
#pragma unroll
        for (int k = 0; k < TriR3::n; ++k)
            far_node(fx, fz, frc2, frc, fic, fic2, flx * (TriR3::s[k] - third), flz * (TriR3::t[k] - third),
                     TriR3::w[k], a);
    }
    monopole_fp64(px, pz, ph, rc2, fic, area, sp, sx, sz, sn);
    const float cf = fic * a.cphi;  // sum w (1/R_k - 1/R_c)
    const float gf = fic * a.gp;    // sum w (1/R_k^3 - 1/R_c^3)
    c.p += cf;
    c.x += fmaf(fx, gf, -a.gx);
    c.z += fmaf(fz, gf, -a.gz);
    c.n = fmaf((float)ph, gf, c.n);
}

// Beyond the quadrupole tier: FP64 monopole plus the FP32 quadrupole term.
template <int KIND>
__device__ __forceinline__ void far_quadrupole(double px, double pz, double ph, double rc2, double lx, double lz,
                                               double area, double &sp, double &sx, double &sz, double &sn,
                                               FarCorr &c)
{
    const float fx = (float)px, fz = (float)pz, fh = (float)ph;
    const float frc2 = (float)rc2;
    const float fic = __builtin_amdgcn_rsqf(frc2);
    const float fic2 = fic * fic;
    const float fic5 = fic2 * fic2 * fic;
    const float flx = (float)lx, flz = (float)lz;
    float mxx, mzz, mpx, mpz;
    if (KIND == 0) {
        mxx = flx * flx * (1.0f / 12.0f);
        mzz = flz * flz * (1.0f / 12.0f);
        mpx = mxx * fx;
        mpz = mzz * fz;
    } else {
        mxx = flx * flx * (1.0f / 18.0f);
        mzz = flz * flz * (1.0f / 18.0f);
        const float mxz = flx * flz * (-1.0f / 36.0f);
        mpx = fmaf(mxx, fx, mxz * fz);
        mpz = fmaf(mxz, fx, mzz * fz);
    }
    const float t = mxx + mzz;
    const float u = fmaf(3.0f, fmaf(fx, mpx, fz * mpz), -frc2 * t);  // 3q - R^2 t
    const float g = fmaf(2.5f * u, fic2, t);
    c.p = fmaf(0.5f * u, fic5, c.p);
    c.x = fmaf(fic5, fmaf(g, fx, -3.0f * mpx), c.x);
    c.z = fmaf(fic5, fmaf(g, fz, -3.0f * mpz), c.z);
    c.n = fmaf(fic5, g * fh, c.n);
    monopole_fp64(px, pz, ph, rc2, fic, area, sp, sx, sz, sn);
}

}  // namespace nebem
