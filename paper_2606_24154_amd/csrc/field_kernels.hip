// field_kernels.hip -- element preparation, field evaluation and influence
// matrix assembly on gfx950.
//
// Work decomposition (both field kernels): one lane owns one observation
// point (an evaluation point, or a collocation row of the matrix) and keeps
// its sums in FP64 registers; a workgroup of 256 lanes (4 wave64) streams the
// derived element records through LDS in tiles, and every lane of the
// workgroup walks the same element of the tile at the same time, so element
// data are wave-uniform: they are read from LDS once per wave and moved to
// scalar registers.  The element kind (rectangle / right triangle) is
// therefore a uniform branch, and the copy loops (lattice translations and
// reflections) are uniform loops.  Each point sums elements in index order
// and copies in lattice order, independent of which other points share its
// wave: results are deterministic and do not depend on the batch a point
// arrives in.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <cmath>

#include "nebem_internal.hpp"
#include "farfield_mixed.hpp"
#include "panel_fp64.hpp"

namespace nebem {

constexpr int kBlock = 256;
constexpr int kTileE = 64;   // elements per LDS tile, evaluation
constexpr int kTileA = 32;   // elements (columns) per workgroup, assembly

// wave-uniform copy of a value held identically by all lanes -> SGPRs
__device__ __forceinline__ double uni(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------------- prep
__global__ __launch_bounds__(kBlock) void k_prep(nebem_panels p, double *__restrict__ drec, int *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= p.n) return;
    const int kind = p.kind[i];
    const int bc = p.bc[i];
    const double ox = p.ox[i], oy = p.oy[i], oz = p.oz[i];
    const double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    const double wx = p.wx[i], wy = p.wy[i], wz = p.wz[i];
    const double lu = sqrt(ux * ux + uy * uy + uz * uz);
    const double lw = sqrt(wx * wx + wy * wy + wz * wz);
    const double uw = ux * wx + uy * wy + uz * wz;
    bool ok = (kind == 0 || kind == 1) && (bc == 0 || bc == 1) && lu > 0.0 && lw > 0.0 &&
              isfinite(lu) && isfinite(lw) && isfinite(ox) && isfinite(oy) && isfinite(oz) &&
              fabs(uw) <= 1e-9 * lu * lw;
    double jump = 0.0;
    if (bc == 1) {
        const double ep = p.eps_pos[i], en = p.eps_neg[i];
        ok = ok && ep > 0.0 && en > 0.0 && ep != en && isfinite(ep) && isfinite(en);
        jump = (ep + en) / (2.0 * kEps0 * (ep - en));
    }
    if (!ok) {
        atomicAdd(&bad[0], 1);
        atomicMin(&bad[1], (int)i);
        return;
    }
    const double e1x = ux / lu, e1y = uy / lu, e1z = uz / lu;
    const double c = wx * e1x + wy * e1y + wz * e1z;
    double vx = wx - c * e1x, vy = wy - c * e1y, vz = wz - c * e1z;
    const double lz = sqrt(vx * vx + vy * vy + vz * vz);
    vx /= lz;
    vy /= lz;
    vz /= lz;
    const double e3x = e1y * vz - e1z * vy, e3y = e1z * vx - e1x * vz, e3z = e1x * vy - e1y * vx;
    const double lx = lu;
    const double hyp = sqrt(lx * lx + lz * lz);
    const double f = kind == 0 ? 0.5 : (1.0 / 3.0);
    double *r = drec + i * R_STRIDE;
    r[R_OX] = ox;
    r[R_OY] = oy;
    r[R_OZ] = oz;
    r[R_E1X] = e1x;
    r[R_E1Y] = e1y;
    r[R_E1Z] = e1z;
    r[R_E2X] = vx;
    r[R_E2Y] = vy;
    r[R_E2Z] = vz;
    r[R_E3X] = e3x;
    r[R_E3Y] = e3y;
    r[R_E3Z] = e3z;
    r[R_LX] = lx;
    r[R_LZ] = lz;
    r[R_HYP] = hyp;
    r[R_IHYP] = 1.0 / hyp;
    r[R_CX] = ox + f * (ux + wx);
    r[R_CY] = oy + f * (uy + wy);
    r[R_CZ] = oz + f * (uz + wz);
    r[R_DIAM] = hyp;
    r[R_AREA] = kind == 0 ? lx * lz : 0.5 * lx * lz;
    r[R_KIND] = (double)kind;
    r[R_JUMP] = jump;
    r[R_BC] = (double)bc;
}

// Triangle pairs: two consecutive right triangles with the same right-angle
// corner, one leg shared (same direction and length) and the other legs
// opposite -- the two halves of a triangle cut at the foot of its altitude,
// as a mesher emits them -- all to 1e-12 relative.  Element i is marked
// kind 2 when its second leg is the shared one (the pair's first triangle
// is i), kind 3 when its first leg is (the first triangle is i + 1).  The
// field kernels then evaluate the two together (rtri_pair_far), taking the
// second triangle's legs as c e2 and -b e1 in the first one's frame: a
// change of its geometry of at most 1e-12 relative, below the far forms'
// own rounding error (~R/D ulps).  Only i's kind is written, so launches
// over any ranges of elements agree.
__device__ __forceinline__ double dist3(const double *a, const double *b, double sb)
{
    const double x = a[0] - sb * b[0], y = a[1] - sb * b[1], z = a[2] - sb * b[2];
    return sqrt(x * x + y * y + z * z);
}

__global__ __launch_bounds__(kBlock) void k_pair_flags(nebem_panels p, double *__restrict__ drec)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i + 1 >= p.n) return;
    if (p.kind[i] != 1 || p.kind[i + 1] != 1) return;
    double *r = drec + i * R_STRIDE;
    const double *q = r + R_STRIDE;
    constexpr double tol = 1e-12;
    if (!(dist3(r + R_OX, q + R_OX, 1.0) <= tol * fmax(r[R_DIAM], q[R_DIAM]))) return;
    if (dist3(r + R_E2X, q + R_E1X, 1.0) <= tol && dist3(r + R_E1X, q + R_E2X, -1.0) <= tol &&
        fabs(r[R_LZ] - q[R_LX]) <= tol * r[R_LZ])
        r[R_KIND] = 2.0;
    else if (dist3(q + R_E2X, r + R_E1X, 1.0) <= tol && dist3(q + R_E1X, r + R_E2X, -1.0) <= tol &&
             fabs(q[R_LZ] - r[R_LX]) <= tol * q[R_LZ])
        r[R_KIND] = 3.0;
}

void launch_prep(const nebem_panels *p, double *drec, int *bad, hipStream_t s)
{
    if (p->n <= 0) return;
    const unsigned g = (unsigned)((p->n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_prep, dim3(g), dim3(kBlock), 0, s, *p, drec, bad);
    hipLaunchKernelGGL(k_pair_flags, dim3(g), dim3(kBlock), 0, s, *p, drec);
}

// ------------------------------------------------------------- one element
// Uniform element data, loaded from an LDS record.
struct Elem {
    double ox, oy, oz, e1x, e1y, e1z, e2x, e2y, e2z, e3x, e3y, e3z;
    double lx, lz, hyp, ihyp;
    double diam, area;
    int kind;
};

__device__ __forceinline__ Elem load_elem(const double *d)
{
    Elem e;
    e.ox = uni(d[R_OX]);
    e.oy = uni(d[R_OY]);
    e.oz = uni(d[R_OZ]);
    e.e1x = uni(d[R_E1X]);
    e.e1y = uni(d[R_E1Y]);
    e.e1z = uni(d[R_E1Z]);
    e.e2x = uni(d[R_E2X]);
    e.e2y = uni(d[R_E2Y]);
    e.e2z = uni(d[R_E2Z]);
    e.e3x = uni(d[R_E3X]);
    e.e3y = uni(d[R_E3Y]);
    e.e3z = uni(d[R_E3Z]);
    e.lx = uni(d[R_LX]);
    e.lz = uni(d[R_LZ]);
    e.hyp = uni(d[R_HYP]);
    e.ihyp = uni(d[R_IHYP]);
    e.diam = uni(d[R_DIAM]);
    e.area = uni(d[R_AREA]);
    e.kind = uni((int)d[R_KIND]);
    return e;
}

// The second triangle of a pair (element records of kind 2 or 3: see
// k_pair_flags): what the pair form needs from its record.
struct PairB {
    double lz, hyp, ihyp, diam, area;
};

__device__ __forceinline__ PairB load_pair_b(const double *d)
{
    PairB f;
    f.lz = uni(d[R_LZ]);
    f.hyp = uni(d[R_HYP]);
    f.ihyp = uni(d[R_IHYP]);
    f.diam = uni(d[R_DIAM]);
    f.area = uni(d[R_AREA]);
    return f;
}

// Sum over lattice translations of one element, local frame; (X0,Z0,H0) is
// the (reflected) point in the element frame for the zero translation, and
// (aX,aZ,aH), (bX,bZ,bH) the lattice vectors in that frame.  `self` zeroes H
// for the zero translation (collocation point on its own element).
// MIXED: copies far enough for a low-order FP32 correction to stay within
// its error budget (R >= 24 D rectangles, 48 D triangles, and never below
// near_factor D) take the FP64 monopole + FP32 correction far field (per
// lane); nearer copies take the exact FP64 closed form, which in that band is
// no more expensive than a higher-order rule would be.
// The exact form is taken per lane in its far-regime evaluation when the
// point is at least kFarDiam diameters from the element's corner o, else in
// the cancellation-free general one; the choice depends on the point alone.
struct MixParams {
    double low2;    // squared distance from which the FP32 low-order rule is used
    double quad2;   // squared distance from which the quadrupole expansion is used
};

template <int KIND, bool MIXED, bool HOLE>
__device__ __forceinline__ void sum_translations(const Elem &e, int n1, int n2, int hole, double X0, double Z0,
                                                 double H0, double aX, double aZ, double aH, double bX, double bZ,
                                                 double bH, bool self, const MixParams &mp, double &sp,
                                                 double &sx, double &sz, double &sn)
{
    const double cxl = KIND == 0 ? 0.5 * e.lx : e.lx * (1.0 / 3.0);
    const double czl = KIND == 0 ? 0.5 * e.lz : e.lz * (1.0 / 3.0);
    const double far2 = (kFarDiam * kFarDiam) * (e.diam * e.diam);
    const double vfar2 = (kVeryFarDiam * kVeryFarDiam) * (e.diam * e.diam);
    FarCorr fc = {0.0f, 0.0f, 0.0f, 0.0f};
    // MIXED: the copies are translated in centroid-relative coordinates,
    // which the far tiers use directly; the exact tiers add the centroid
    // offset back
    if (MIXED) {
        X0 -= cxl;
        Z0 -= czl;
    }
#pragma unroll 1
    for (int i1 = -n1; i1 <= n1; ++i1) {
        const double f1 = -(double)i1;
        const double X1 = fma(f1, aX, X0), Z1 = fma(f1, aZ, Z0), H1 = fma(f1, aH, H0);
        // HOLE: a row that crosses the hole runs as two ranges of i2, so the
        // inner loop itself carries no test for it
        const bool cut = HOLE && abs(i1) <= hole;
#pragma unroll 1
        for (int seg = 0; seg <= (int)cut; ++seg) {
            const int i2a = seg == 0 ? -n2 : hole + 1;
            const int i2b = (cut && seg == 0) ? -hole - 1 : n2;
#pragma unroll 1
            for (int i2 = i2a; i2 <= i2b; ++i2) {
                const double f2 = -(double)i2;
                double X = fma(f2, bX, X1), Z = fma(f2, bZ, Z1);
                double H = fma(f2, bH, H1);
                H = (self && i1 == 0 && i2 == 0) ? 0.0 : H;
                if (MIXED) {
                    const double rc2 = fma(X, X, fma(Z, Z, H * H));
                    if (rc2 >= mp.quad2) {
                        far_quadrupole<KIND>(X, Z, H, rc2, e.lx, e.lz, e.area, sp, sx, sz, sn, fc);
                        continue;
                    }
                    if (rc2 >= mp.low2) {
                        far_mixed<KIND>(X, Z, H, rc2, e.lx, e.lz, e.area, sp, sx, sz, sn, fc);
                        continue;
                    }
                    X += cxl;
                    Z += czl;
                }
                Kern k;
                const double r0sq = fma(X, X, fma(Z, Z, H * H));
                if (r0sq >= vfar2) {  // far forms return the potential added to sp
                    if (KIND == 0)
                        k = rect_far<true>(X, H, Z, e.lx, e.lz, r0sq, sp);
                    else
                        k = rtri_far<true>(X, H, Z, e.lx, e.lz, e.hyp, r0sq, sp);
                } else if (r0sq >= far2) {
                    if (KIND == 0)
                        k = rect_far<false>(X, H, Z, e.lx, e.lz, r0sq, sp);
                    else
                        k = rtri_far<false>(X, H, Z, e.lx, e.lz, e.hyp, r0sq, sp);
                } else {
                    if (KIND == 0)
                        k = rect_fp64(X, H, Z, e.lx, e.lz, r0sq);
                    else
                        k = rtri_fp64(X, H, Z, e.lx, e.lz, e.hyp, e.ihyp, r0sq);
                    k.phi += sp;
                }
                sp = k.phi;
                sx += k.ex;
                sz += k.ez;
                sn += k.en;
            }
        }
    }
    if (MIXED) {
        sp = fma(e.area, (double)fc.p, sp);
        sx = fma(e.area, (double)fc.x, sx);
        sz = fma(e.area, (double)fc.z, sz);
        sn = fma(e.area, (double)fc.n, sn);
    }
}

// phi', E' (global frame) of one element with all its copies at P.
template <bool MIXED, bool HOLE = false>
__device__ __forceinline__ void element_copies(const Elem &e, const ImgArgs &img, double Px, double Py, double Pz,
                                               bool self, double near_factor, double &ophi, double &oex,
                                               double &oey, double &oez)
{
    MixParams mp;
    if (MIXED) {
        const double nd = near_factor * e.diam;
        const double ld = fmax(nd, (e.kind == 0 ? 24.0 : 48.0) * e.diam);
        const double qd = fmax(nd, (e.kind == 0 ? 32.0 : 96.0) * e.diam);
        mp.low2 = ld * ld;
        mp.quad2 = qd * qd;
    }
    ophi = oex = oey = oez = 0.0;
    for (int r = 0; r < img.nref; ++r) {
        const int ax = img.axes[r];
        const double Qx = (ax & 1) ? 2.0 * img.mpos[0] - Px : Px;
        const double Qy = (ax & 2) ? 2.0 * img.mpos[1] - Py : Py;
        const double Qz = (ax & 4) ? 2.0 * img.mpos[2] - Pz : Pz;
        const double rx = Qx - e.ox, ry = Qy - e.oy, rz = Qz - e.oz;
        const double X0 = rx * e.e1x + ry * e.e1y + rz * e.e1z;
        const double Z0 = rx * e.e2x + ry * e.e2y + rz * e.e2z;
        const double H0 = rx * e.e3x + ry * e.e3y + rz * e.e3z;
        const double *a = img.a1[r], *b = img.a2[r];
        const double aX = a[0] * e.e1x + a[1] * e.e1y + a[2] * e.e1z;
        const double aZ = a[0] * e.e2x + a[1] * e.e2y + a[2] * e.e2z;
        const double aH = a[0] * e.e3x + a[1] * e.e3y + a[2] * e.e3z;
        const double bX = b[0] * e.e1x + b[1] * e.e1y + b[2] * e.e1z;
        const double bZ = b[0] * e.e2x + b[1] * e.e2y + b[2] * e.e2z;
        const double bH = b[0] * e.e3x + b[1] * e.e3y + b[2] * e.e3z;
        double sp = 0.0, sx = 0.0, sz = 0.0, sn = 0.0;
        const bool s = self && r == 0;
        if (e.kind == 0)
            sum_translations<0, MIXED, HOLE>(e, img.n1, img.n2, img.hole, X0, Z0, H0, aX, aZ, aH, bX, bZ, bH, s, mp, sp,
                                       sx, sz, sn);
        else
            sum_translations<1, MIXED, HOLE>(e, img.n1, img.n2, img.hole, X0, Z0, H0, aX, aZ, aH, bX, bZ, bH, s, mp, sp,
                                       sx, sz, sn);
        double gx = sx * e.e1x + sz * e.e2x + sn * e.e3x;
        double gy = sx * e.e1y + sz * e.e2y + sn * e.e3y;
        double gz = sx * e.e1z + sz * e.e2z + sn * e.e3z;
        gx = (ax & 1) ? -gx : gx;
        gy = (ax & 2) ? -gy : gy;
        gz = (ax & 4) ? -gz : gz;
        const double par = img.parity[r];
        ophi += par * sp;
        oex += par * gx;
        oey += par * gy;
        oez += par * gz;
    }
}

// Sum over lattice translations of a triangle pair (FP64 evaluation only),
// in the first triangle's frame: the second triangle's legs are c = e.lz
// along e2 and b = f.lz along -e1 (the geometry the pair flag was tested
// for, within 1e-12 of its own record), so its frame is (e2, -e1, e3) and
// its sums come back in that frame.  Tiers as in sum_translations, by the
// distance from the shared corner in units of the larger diameter; below
// the far regime each triangle takes the general form.
template <bool HOLE>
__device__ __forceinline__ void sum_translations_pair(const Elem &e, const PairB &f, int n1, int n2, int hole,
                                                      double X0, double Z0, double H0, double aX, double aZ,
                                                      double aH, double bX, double bZ, double bH, double (&s1)[4],
                                                      double (&s2)[4])
{
    const double a = e.lx, c = e.lz, b = f.lz;
    const double dp = fmax(e.diam, f.diam);
    const double far2 = (kFarDiam * kFarDiam) * (dp * dp);
    const double vfar2 = (kVeryFarDiam * kVeryFarDiam) * (dp * dp);
#pragma unroll 1
    for (int i1 = -n1; i1 <= n1; ++i1) {
        const double f1 = -(double)i1;
        const double X1 = fma(f1, aX, X0), Z1 = fma(f1, aZ, Z0), H1 = fma(f1, aH, H0);
        const bool cut = HOLE && abs(i1) <= hole;
#pragma unroll 1
        for (int seg = 0; seg <= (int)cut; ++seg) {
            const int i2a = seg == 0 ? -n2 : hole + 1;
            const int i2b = (cut && seg == 0) ? -hole - 1 : n2;
#pragma unroll 1
            for (int i2 = i2a; i2 <= i2b; ++i2) {
                const double f2 = -(double)i2;
                const double X = fma(f2, bX, X1), Z = fma(f2, bZ, Z1);
                const double H = fma(f2, bH, H1);
                const double r0sq = fma(X, X, fma(Z, Z, H * H));
                Kern k1, k2;
                if (r0sq >= vfar2) {  // far forms return the potentials added to the sums
                    rtri_pair_far<true>(X, H, Z, a, b, c, e.hyp, f.hyp, r0sq, s1[0], s2[0], k1, k2);
                } else if (r0sq >= far2) {
                    rtri_pair_far<false>(X, H, Z, a, b, c, e.hyp, f.hyp, r0sq, s1[0], s2[0], k1, k2);
                } else {
                    k1 = rtri_fp64(X, H, Z, a, c, e.hyp, e.ihyp, r0sq);
                    k2 = rtri_fp64(Z, H, -X, c, b, f.hyp, f.ihyp, r0sq);
                    k1.phi += s1[0];
                    k2.phi += s2[0];
                }
                s1[0] = k1.phi;
                s1[1] += k1.ex;
                s1[2] += k1.ez;
                s1[3] += k1.en;
                s2[0] = k2.phi;
                s2[1] += k2.ex;
                s2[2] += k2.ez;
                s2[3] += k2.en;
            }
        }
    }
}

// phi', E' (global frame) of both triangles of a pair with all their copies
// at P: o1 for the first, o2 for the second.
template <bool HOLE>
__device__ __forceinline__ void element_pair_copies(const Elem &e, const PairB &f, const ImgArgs &img, double Px,
                                                    double Py, double Pz, double (&o1)[4], double (&o2)[4])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) o1[c] = o2[c] = 0.0;
    for (int r = 0; r < img.nref; ++r) {
        const int ax = img.axes[r];
        const double Qx = (ax & 1) ? 2.0 * img.mpos[0] - Px : Px;
        const double Qy = (ax & 2) ? 2.0 * img.mpos[1] - Py : Py;
        const double Qz = (ax & 4) ? 2.0 * img.mpos[2] - Pz : Pz;
        const double rx = Qx - e.ox, ry = Qy - e.oy, rz = Qz - e.oz;
        const double X0 = rx * e.e1x + ry * e.e1y + rz * e.e1z;
        const double Z0 = rx * e.e2x + ry * e.e2y + rz * e.e2z;
        const double H0 = rx * e.e3x + ry * e.e3y + rz * e.e3z;
        const double *a = img.a1[r], *b = img.a2[r];
        const double aX = a[0] * e.e1x + a[1] * e.e1y + a[2] * e.e1z;
        const double aZ = a[0] * e.e2x + a[1] * e.e2y + a[2] * e.e2z;
        const double aH = a[0] * e.e3x + a[1] * e.e3y + a[2] * e.e3z;
        const double bX = b[0] * e.e1x + b[1] * e.e1y + b[2] * e.e1z;
        const double bZ = b[0] * e.e2x + b[1] * e.e2y + b[2] * e.e2z;
        const double bH = b[0] * e.e3x + b[1] * e.e3y + b[2] * e.e3z;
        double s1[4] = {0.0, 0.0, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.0, 0.0};
        sum_translations_pair<HOLE>(e, f, img.n1, img.n2, img.hole, X0, Z0, H0, aX, aZ, aH, bX, bZ, bH, s1, s2);
        // first triangle: frame (e1, e2, e3); second: (e2, -e1, e3)
        double g1x = s1[1] * e.e1x + s1[2] * e.e2x + s1[3] * e.e3x;
        double g1y = s1[1] * e.e1y + s1[2] * e.e2y + s1[3] * e.e3y;
        double g1z = s1[1] * e.e1z + s1[2] * e.e2z + s1[3] * e.e3z;
        double g2x = s2[1] * e.e2x - s2[2] * e.e1x + s2[3] * e.e3x;
        double g2y = s2[1] * e.e2y - s2[2] * e.e1y + s2[3] * e.e3y;
        double g2z = s2[1] * e.e2z - s2[2] * e.e1z + s2[3] * e.e3z;
        g1x = (ax & 1) ? -g1x : g1x;
        g1y = (ax & 2) ? -g1y : g1y;
        g1z = (ax & 4) ? -g1z : g1z;
        g2x = (ax & 1) ? -g2x : g2x;
        g2y = (ax & 2) ? -g2y : g2y;
        g2z = (ax & 4) ? -g2z : g2z;
        const double par = img.parity[r];
        o1[0] += par * s1[0];
        o1[1] += par * g1x;
        o1[2] += par * g1y;
        o1[3] += par * g1z;
        o2[0] += par * s2[0];
        o2[1] += par * g2x;
        o2[2] += par * g2y;
        o2[3] += par * g2z;
    }
}

// ----------------------------------------------------- mixed-path pairs
// In the mixed path a triangle pair far enough away is taken as one charge
// distribution: the sigma-weighted monopole (FP64), dipole and second
// moments (FP32) of both triangles about the centroid c0 of the whole
// triangle they came from.  In the first triangle's frame the pair has
// vertices o, A = o + a e1, C = o + c e2, B = o - b e1; its triangles'
// centroids lie (b/3, 0) and (-a/3, 0) from c0 = o + ((a - b)/3, c/3), so
// with charges w1 = sigma1 A1, w2 = sigma2 A2 the dipole is
// ((w1 b - w2 a)/3, 0) and the second moments are the triangles' central
// ones (right triangle per unit area: lx^2/18, lz^2/18, -lx lz/36 in its
// own frame; the second triangle's frame is (e2, -e1)) moved to c0.  The
// expansion is the multipole series of the single-triangle quadrupole tier
// (farfield_mixed.hpp) with the dipole term added; it is used from 96
// diameters of the whole triangle (a + b, which bounds every vertex's
// distance from c0 by (a + b) 2/3), where the truncation error relative to
// |w1| + |w2| is at most the single triangle's at 96 of its own diameters.
// Nearer copies take each triangle's own mixed tiers.  One such copy costs
// about what one triangle's quadrupole copy costs.
// The FP32 moments are carried in units of sc = |w1| + |w2| (so that their
// range does not depend on the densities' scale), and the FP32 corrections
// are multiplied by sc once, in FP64, after the copies.
template <int K>
struct PairMoments {
    double q[K], sc[K];                   // w1 + w2; |w1| + |w2|
    float dx[K], mxx[K], mzz[K], mxz[K];  // dipole (along e1), second moments, in units of sc
};

template <int K>
__device__ __forceinline__ PairMoments<K> pair_moments(double a, double b, double c, double area1, double area2,
                                                       const double (&sg1)[K], const double (&sg2)[K])
{
    PairMoments<K> m;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double v1 = sg1[k] * area1, v2 = sg2[k] * area2;
        m.q[k] = v1 + v2;
        const double sc = fabs(v1) + fabs(v2);
        m.sc[k] = sc > 0.0 ? sc : 1.0;
        const double w1 = v1 / m.sc[k], w2 = v2 / m.sc[k];
        m.dx[k] = (float)((w1 * b - w2 * a) * (1.0 / 3.0));
        m.mxx[k] = (float)(w1 * (a * a * (1.0 / 18.0) + b * b * (1.0 / 9.0)) +
                           w2 * (b * b * (1.0 / 18.0) + a * a * (1.0 / 9.0)));
        m.mzz[k] = (float)((w1 + w2) * (c * c * (1.0 / 18.0)));
        m.mxz[k] = (float)((w2 * b - w1 * a) * (c * (1.0 / 36.0)));
    }
    return m;
}

// One copy of the pair as one distribution at p = P - c0 (FP64, the first
// triangle's frame), rc2 = |p|^2: sigma-weighted monopole into s[k] (FP64),
// dipole + quadrupole corrections, in units of m.sc[k], into fc[k] (FP32).
template <int K>
__device__ __forceinline__ void pair_far_moments(double px, double pz, double ph, double rc2,
                                                 const PairMoments<K> &m, double (&s)[K][4], FarCorr (&fc)[K])
{
    const float fx = (float)px, fz = (float)pz, fh = (float)ph;
    const float frc2 = (float)rc2;
    const float fic = __builtin_amdgcn_rsqf(frc2);
    const float fic2 = fic * fic;
    const float fic3 = fic2 * fic;
    const float fic5 = fic3 * fic2;
    double ir = (double)fic;
    ir = ir * (1.5 - 0.5 * rc2 * ir * ir);
    const double ir2 = ir * ir;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double air = m.q[k] * ir;
        const double air3 = air * ir2;
        s[k][0] += air;
        s[k][1] = fma(air3, px, s[k][1]);
        s[k][2] = fma(air3, pz, s[k][2]);
        s[k][3] = fma(air3, ph, s[k][3]);
        const float mpx = fmaf(m.mxx[k], fx, m.mxz[k] * fz);
        const float mpz = fmaf(m.mxz[k], fx, m.mzz[k] * fz);
        const float t = m.mxx[k] + m.mzz[k];
        const float u = fmaf(3.0f, fmaf(fx, mpx, fz * mpz), -frc2 * t);  // 3q - R^2 t
        const float dpx = m.dx[k] * fx;                                   // d.p
        const float G = fmaf(3.0f, dpx, fmaf(2.5f * u, fic2, t));  // p coefficient (x fic5): quadrupole g + dipole 3 d.p
        fc[k].p += fmaf(0.5f * u, fic5, dpx * fic3);
        fc[k].x += fmaf(fic5, fmaf(G, fx, -3.0f * mpx), -m.dx[k] * fic3);
        fc[k].z = fmaf(fic5, fmaf(G, fz, -3.0f * mpz), fc[k].z);
        fc[k].n = fmaf(fic5, G * fh, fc[k].n);
    }
}

// One copy of one right triangle in the mixed path, unit density, at
// centroid-relative (Xc, Zc, H) in its own frame: the tiers of
// sum_translations<1, true>.
__device__ __forceinline__ void tri_copy_mixed(double Xc, double Zc, double H, double lx, double lz, double hyp,
                                               double ihyp, double area, const MixParams &mp, double far2,
                                               double vfar2, double (&s)[4], FarCorr &fc)
{
    const double rc2 = fma(Xc, Xc, fma(Zc, Zc, H * H));
    if (rc2 >= mp.quad2) {
        far_quadrupole<1>(Xc, Zc, H, rc2, lx, lz, area, s[0], s[1], s[2], s[3], fc);
        return;
    }
    if (rc2 >= mp.low2) {
        far_mixed<1>(Xc, Zc, H, rc2, lx, lz, area, s[0], s[1], s[2], s[3], fc);
        return;
    }
    const double X = Xc + lx * (1.0 / 3.0), Z = Zc + lz * (1.0 / 3.0);
    const double r0sq = fma(X, X, fma(Z, Z, H * H));
    Kern k;
    if (r0sq >= vfar2) {
        k = rtri_far<true>(X, H, Z, lx, lz, hyp, r0sq, s[0]);
    } else if (r0sq >= far2) {
        k = rtri_far<false>(X, H, Z, lx, lz, hyp, r0sq, s[0]);
    } else {
        k = rtri_fp64(X, H, Z, lx, lz, hyp, ihyp, r0sq);
        k.phi += s[0];
    }
    s[0] = k.phi;
    s[1] += k.ex;
    s[2] += k.ez;
    s[3] += k.en;
}

__device__ __forceinline__ MixParams mix_params(double near_factor, double diam, double low_d, double quad_d)
{
    MixParams mp;
    const double nd = near_factor * diam;
    const double ld = fmax(nd, low_d * diam), qd = fmax(nd, quad_d * diam);
    mp.low2 = ld * ld;
    mp.quad2 = qd * qd;
    return mp;
}

// phi', E' (global frame) of a triangle pair with all its copies at P in the
// mixed path, weighted by each column's densities (sg1, sg2): out[k].
template <int K, bool HOLE>
__device__ __forceinline__ void element_pair_copies_mixed(const Elem &e, const PairB &f, const double (&sg1)[K],
                                                          const double (&sg2)[K], const ImgArgs &img,
                                                          double near_factor, double Px, double Py, double Pz,
                                                          double (&out)[K][4])
{
    const double a = e.lx, c = e.lz, b = f.lz;
    const PairMoments<K> pm = pair_moments<K>(a, b, c, e.area, f.area, sg1, sg2);
    const MixParams mp1 = mix_params(near_factor, e.diam, 48.0, 96.0);
    const MixParams mp2 = mix_params(near_factor, f.diam, 48.0, 96.0);
    const MixParams mpp = mix_params(near_factor, a + b, 48.0, 96.0);
    const double far1 = (kFarDiam * kFarDiam) * (e.diam * e.diam), vfar1 = (kVeryFarDiam * kVeryFarDiam) * (e.diam * e.diam);
    const double far2 = (kFarDiam * kFarDiam) * (f.diam * f.diam), vfar2 = (kVeryFarDiam * kVeryFarDiam) * (f.diam * f.diam);
    const double c0x = (a - b) * (1.0 / 3.0), c0z = c * (1.0 / 3.0);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) out[k][q] = 0.0;
    for (int r = 0; r < img.nref; ++r) {
        const int ax = img.axes[r];
        const double Qx = (ax & 1) ? 2.0 * img.mpos[0] - Px : Px;
        const double Qy = (ax & 2) ? 2.0 * img.mpos[1] - Py : Py;
        const double Qz = (ax & 4) ? 2.0 * img.mpos[2] - Pz : Pz;
        const double rx = Qx - e.ox, ry = Qy - e.oy, rz = Qz - e.oz;
        // coordinates relative to c0
        const double X0 = rx * e.e1x + ry * e.e1y + rz * e.e1z - c0x;
        const double Z0 = rx * e.e2x + ry * e.e2y + rz * e.e2z - c0z;
        const double H0 = rx * e.e3x + ry * e.e3y + rz * e.e3z;
        const double *av = img.a1[r], *bv = img.a2[r];
        const double aX = av[0] * e.e1x + av[1] * e.e1y + av[2] * e.e1z;
        const double aZ = av[0] * e.e2x + av[1] * e.e2y + av[2] * e.e2z;
        const double aH = av[0] * e.e3x + av[1] * e.e3y + av[2] * e.e3z;
        const double bX = bv[0] * e.e1x + bv[1] * e.e1y + bv[2] * e.e1z;
        const double bZ = bv[0] * e.e2x + bv[1] * e.e2y + bv[2] * e.e2z;
        const double bH = bv[0] * e.e3x + bv[1] * e.e3y + bv[2] * e.e3z;
        double sp[K][4];  // sigma-weighted, first triangle's frame
        FarCorr fp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            sp[k][0] = sp[k][1] = sp[k][2] = sp[k][3] = 0.0;
            fp[k] = {0.0f, 0.0f, 0.0f, 0.0f};
        }
        double s1[4] = {0.0, 0.0, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.0, 0.0};  // unit density, own frames
        FarCorr f1 = {0.0f, 0.0f, 0.0f, 0.0f}, f2 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
        for (int i1 = -img.n1; i1 <= img.n1; ++i1) {
            const double g1 = -(double)i1;
            const double X1 = fma(g1, aX, X0), Z1 = fma(g1, aZ, Z0), H1 = fma(g1, aH, H0);
            const bool cut = HOLE && abs(i1) <= img.hole;
#pragma unroll 1
            for (int seg = 0; seg <= (int)cut; ++seg) {
                const int i2a = seg == 0 ? -img.n2 : img.hole + 1;
                const int i2b = (cut && seg == 0) ? -img.hole - 1 : img.n2;
#pragma unroll 1
                for (int i2 = i2a; i2 <= i2b; ++i2) {
                    const double g2 = -(double)i2;
                    const double X = fma(g2, bX, X1), Z = fma(g2, bZ, Z1), H = fma(g2, bH, H1);
                    const double rc2 = fma(X, X, fma(Z, Z, H * H));
                    if (rc2 >= mpp.quad2) {
                        pair_far_moments<K>(X, Z, H, rc2, pm, sp, fp);
                        continue;
                    }
                    // each triangle on its own: corner-relative (X + c0x, Z + c0z);
                    // the second one's frame (e2, -e1): (Z + c0z, -(X + c0x))
                    const double Xo = X + c0x, Zo = Z + c0z;
                    tri_copy_mixed(Xo - a * (1.0 / 3.0), Zo - c * (1.0 / 3.0), H, a, c, e.hyp, e.ihyp, e.area, mp1,
                                   far1, vfar1, s1, f1);
                    tri_copy_mixed(Zo - c * (1.0 / 3.0), -Xo - b * (1.0 / 3.0), H, c, b, f.hyp, f.ihyp, f.area, mp2,
                                   far2, vfar2, s2, f2);
                }
            }
        }
        // unit-density sums with their FP32 corrections, the second
        // triangle's turned into the first one's frame (e1 = -e2', e2 = e1')
        const double u1[4] = {fma(e.area, (double)f1.p, s1[0]), fma(e.area, (double)f1.x, s1[1]),
                              fma(e.area, (double)f1.z, s1[2]), fma(e.area, (double)f1.n, s1[3])};
        const double u2[4] = {fma(f.area, (double)f2.p, s2[0]), -fma(f.area, (double)f2.z, s2[2]),
                              fma(f.area, (double)f2.x, s2[1]), fma(f.area, (double)f2.n, s2[3])};
        const double par = img.parity[r];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double l[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) l[q] = fma(sg2[k], u2[q], fma(sg1[k], u1[q], sp[k][q]));
            l[0] = fma(pm.sc[k], (double)fp[k].p, l[0]);
            l[1] = fma(pm.sc[k], (double)fp[k].x, l[1]);
            l[2] = fma(pm.sc[k], (double)fp[k].z, l[2]);
            l[3] = fma(pm.sc[k], (double)fp[k].n, l[3]);
            double gx = l[1] * e.e1x + l[2] * e.e2x + l[3] * e.e3x;
            double gy = l[1] * e.e1y + l[2] * e.e2y + l[3] * e.e3y;
            double gz = l[1] * e.e1z + l[2] * e.e2z + l[3] * e.e3z;
            gx = (ax & 1) ? -gx : gx;
            gy = (ax & 2) ? -gy : gy;
            gz = (ax & 4) ? -gz : gz;
            out[k][0] += par * l[0];
            out[k][1] += par * gx;
            out[k][2] += par * gy;
            out[k][3] += par * gz;
        }
    }
}

// -------------------------------------------------------------- evaluation
// One workgroup's share of an evaluation: points [base, base + BS) of the
// m points, all n elements (records drec, densities sigma) and their copies,
// FP64 sums per lane; outputs scaled by `scale`.
template <bool MIXED, int BS, bool HOLE = false>
__device__ __forceinline__ void eval_block(const double *__restrict__ drec, const double *__restrict__ sigma, int n,
                                           const ImgArgs &img, double near_factor, const double *__restrict__ px,
                                           const double *__restrict__ py, const double *__restrict__ pz, int m,
                                           int base_pt, double scale, double *__restrict__ phi,
                                           double *__restrict__ ex, double *__restrict__ ey,
                                           double *__restrict__ ez)
{
    __shared__ double t_rec[kTileE * R_STRIDE];
    __shared__ double t_sig[kTileE];
    const int i = base_pt + threadIdx.x;
    const bool act = i < m;
    const double Px = act ? px[i] : 0.0;
    const double Py = act ? py[i] : 0.0;
    const double Pz = act ? pz[i] : 0.0;
    double aphi = 0.0, aex = 0.0, aey = 0.0, aez = 0.0;
    for (int base = 0; base < n; base += kTileE) {
        const int cnt = min(kTileE, n - base);
        __syncthreads();
        for (int k = threadIdx.x; k < cnt * R_STRIDE; k += BS) t_rec[k] = drec[(size_t)base * R_STRIDE + k];
        for (int k = threadIdx.x; k < cnt; k += BS) t_sig[k] = sigma[base + k];
        __syncthreads();
        for (int p = 0; p < cnt; ++p) {
            const Elem e = load_elem(t_rec + p * R_STRIDE);
            if (MIXED && e.kind >= 2 && p + 1 < cnt) {
                // a triangle pair inside this tile, sigma-weighted in one pass
                const int q1 = e.kind == 2 ? p : p + 1, q2 = e.kind == 2 ? p + 1 : p;
                const double sg1[1] = {uni(t_sig[q1])}, sg2[1] = {uni(t_sig[q2])};
                double c[1][4];
                element_pair_copies_mixed<1, HOLE>(load_elem(t_rec + q1 * R_STRIDE), load_pair_b(t_rec + q2 * R_STRIDE),
                                                   sg1, sg2, img, near_factor, Px, Py, Pz, c);
                aphi += c[0][0];
                aex += c[0][1];
                aey += c[0][2];
                aez += c[0][3];
                ++p;
                continue;
            }
            if (!MIXED && e.kind >= 2 && p + 1 < cnt) {
                // a triangle pair inside this tile: both in one pass (c1 for
                // element p, c2 for p + 1, whichever is the pair's first)
                const int q1 = e.kind == 2 ? p : p + 1, q2 = e.kind == 2 ? p + 1 : p;
                double c[2][4];
                element_pair_copies<HOLE>(load_elem(t_rec + q1 * R_STRIDE), load_pair_b(t_rec + q2 * R_STRIDE), img,
                                          Px, Py, Pz, c[q1 - p], c[q2 - p]);
                const double(&c1)[4] = c[0], (&c2)[4] = c[1];
                const double s1 = uni(t_sig[p]), s2 = uni(t_sig[p + 1]);
                aphi = fma(s2, c2[0], fma(s1, c1[0], aphi));
                aex = fma(s2, c2[1], fma(s1, c1[1], aex));
                aey = fma(s2, c2[2], fma(s1, c1[2], aey));
                aez = fma(s2, c2[3], fma(s1, c1[3], aez));
                ++p;
                continue;
            }
            double cp, cx, cy, cz;
            element_copies<MIXED, HOLE>(e, img, Px, Py, Pz, false, near_factor, cp, cx, cy, cz);
            const double sg = uni(t_sig[p]);
            aphi = fma(sg, cp, aphi);
            aex = fma(sg, cx, aex);
            aey = fma(sg, cy, aey);
            aez = fma(sg, cz, aez);
        }
    }
    if (act) {
        if (phi) phi[i] = scale * aphi;
        if (ex) ex[i] = scale * aex;
        if (ey) ey[i] = scale * aey;
        if (ez) ez[i] = scale * aez;
    }
}

// Element segments.  Every evaluation path (stateless, session, ordered,
// several-column, serving) splits a geometry's elements into the same
// contiguous segments of about kSegWork interactions per point, evaluates
// each (point, segment) pair as an independent unit and adds the segments'
// partial sums in segment order.  The plan depends on the element count and
// the copies only, so a point's result does not depend on how many other
// points share its launch; and a launch of a few hundred thousand points
// over tens of thousands of elements still has ~10^5 workgroups, so its last
// round of waves is a small share of it (one workgroup per 256 points over
// all elements would leave a 200 000-point launch at 1.5 rounds).
int64_t img_copies(const ImgArgs &img)
{
    int64_t t = (int64_t)(2 * img.n1 + 1) * (2 * img.n2 + 1);
    if (img.hole >= 0) {
        const int64_t h1 = img.hole < img.n1 ? img.hole : img.n1;
        const int64_t h2 = img.hole < img.n2 ? img.hole : img.n2;
        t -= (2 * h1 + 1) * (2 * h2 + 1);
    }
    return (int64_t)img.nref * t;
}

SegPlan seg_plan(int64_t n, const ImgArgs &img)
{
    SegPlan p = {1, (int)(n > 0 ? n : 1)};
    if (n <= 0) return p;
    const double per_pt = (double)n * (double)img_copies(img);
    int nseg = (int)(per_pt / kSegWork + 0.5);
    nseg = nseg < 1 ? 1 : (nseg > kMaxSeg ? kMaxSeg : nseg);
    if (nseg > n) nseg = (int)n;
    p.segsz = (int)((n + nseg - 1) / nseg);
    p.nseg = (int)((n + p.segsz - 1) / p.segsz);
    return p;
}

// FP64: the default allocation (about 250 VGPRs, two waves per SIMD) keeps every
// value in registers; a three-wave target made the allocator spill part of
// the per-element setup to scratch (10.6 GB of HBM writes per 10^6-point
// launch) for no measurable gain.  HOLE: img.hole is honoured (a separate
// instantiation, so the plain launch carries no test for it).
// Grid: x over blocks of kBlock points, y over element segments of segsz
// elements; segment y writes its sums (times `scale`) at outputs + y * seg_stride.
template <bool HOLE>
__global__ __launch_bounds__(kBlock) void k_eval_fp64(
    const double *__restrict__ drec, const double *__restrict__ sigma, int n, int segsz, ImgArgs img,
    double near_factor, const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ pz,
    int m, double scale, double *__restrict__ phi, double *__restrict__ ex, double *__restrict__ ey,
    double *__restrict__ ez, int64_t seg_stride)
{
    const int e0 = blockIdx.y * segsz;
    const size_t so = (size_t)blockIdx.y * (size_t)seg_stride;
    eval_block<false, kBlock, HOLE>(drec + (size_t)e0 * R_STRIDE, sigma + e0, min(segsz, n - e0), img, near_factor,
                                    px, py, pz, m, blockIdx.x * kBlock, scale, phi ? phi + so : nullptr,
                                    ex ? ex + so : nullptr, ey ? ey + so : nullptr, ez ? ez + so : nullptr);
}

// Mixed: two waves per SIMD (the triangle-pair path holds two triangles'
// unit-density sums and the pair's weighted ones at once; at three waves it
// spilled inside the copy loop).
template <bool HOLE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_eval_mixed(
    const double *__restrict__ drec, const double *__restrict__ sigma, int n, int segsz, ImgArgs img,
    double near_factor, const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ pz,
    int m, double scale, double *__restrict__ phi, double *__restrict__ ex, double *__restrict__ ey,
    double *__restrict__ ez, int64_t seg_stride)
{
    const int e0 = blockIdx.y * segsz;
    const size_t so = (size_t)blockIdx.y * (size_t)seg_stride;
    eval_block<true, kBlock, HOLE>(drec + (size_t)e0 * R_STRIDE, sigma + e0, min(segsz, n - e0), img, near_factor,
                                   px, py, pz, m, blockIdx.x * kBlock, scale, phi ? phi + so : nullptr,
                                   ex ? ex + so : nullptr, ey ? ey + so : nullptr, ez ? ez + so : nullptr);
}

void launch_eval_seg(const double *drec, const double *sigma, int64_t n, const SegPlan &sp, const ImgArgs &img,
                     int mixed, double near_factor, const double *px, const double *py, const double *pz, int64_t m,
                     double scale, double *phi, double *ex, double *ey, double *ez, int64_t seg_stride, hipStream_t s)
{
    if (m <= 0 || n <= 0) return;
    const dim3 g((unsigned)((m + kBlock - 1) / kBlock), (unsigned)sp.nseg);
    const bool hole = img.hole >= 0;
    auto k = mixed ? (hole ? k_eval_mixed<true> : k_eval_mixed<false>)
                   : (hole ? k_eval_fp64<true> : k_eval_fp64<false>);
    hipLaunchKernelGGL(k, g, dim3(kBlock), 0, s, drec, sigma, (int)n, sp.segsz, img, near_factor, px, py, pz, (int)m,
                       scale, phi, ex, ey, ez, seg_stride);
}

// out[c][i] += add[c m + i] for the non-null outputs
__global__ __launch_bounds__(kBlock) void k_add4(const double *__restrict__ add, int m, double *__restrict__ o0,
                                                 double *__restrict__ o1, double *__restrict__ o2,
                                                 double *__restrict__ o3)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const size_t mm = (size_t)m;
    if (o0) o0[i] += add[i];
    if (o1) o1[i] += add[mm + i];
    if (o2) o2[i] += add[2 * mm + i];
    if (o3) o3[i] += add[3 * mm + i];
}

void launch_add4(const double *add, int64_t m, double *o0, double *o1, double *o2, double *o3, hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_add4, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, add, (int)m, o0, o1,
                       o2, o3);
}

// Primitive-averaged densities (Adaptive Modelling): sbar[p] = (sum of
// sigma_j A_j over the elements j with map[j] == p, in element order) / A_p.
// The elements are first sorted by primitive (stable radix sort of
// (map[j], j)); then one lane per primitive finds its run by binary search
// and sums it in order -- O(n log n) work instead of every lane scanning all
// n elements, the same sums bit for bit.  *bad is set when a map entry is
// outside [0, np) (such an element is sorted past every primitive).
__global__ __launch_bounds__(kBlock) void k_prim_keys(const int32_t *__restrict__ map, int n, int np,
                                                      unsigned *__restrict__ key, int *__restrict__ idx,
                                                      int *__restrict__ bad)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int mj = map[j];
    const bool ok = mj >= 0 && mj < np;
    if (!ok) bad[0] = 1;
    key[j] = ok ? (unsigned)mj : (unsigned)np;
    idx[j] = j;
}

__device__ __forceinline__ int lower_bound_u(const unsigned *__restrict__ a, int n, unsigned v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_prim_density(const double *__restrict__ drec,
                                                         const double *__restrict__ sigma,
                                                         const unsigned *__restrict__ key,
                                                         const int *__restrict__ idx, int n,
                                                         const double *__restrict__ prec, int np,
                                                         double *__restrict__ sbar)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const int s0 = lower_bound_u(key, n, (unsigned)p), s1 = lower_bound_u(key, n, (unsigned)p + 1u);
    double q = 0.0;
    for (int s = s0; s < s1; ++s) {
        const int j = idx[s];
        q = fma(sigma[j], drec[(size_t)j * R_STRIDE + R_AREA], q);
    }
    sbar[p] = q / prec[(size_t)p * R_STRIDE + R_AREA];
}

size_t prim_density_workspace(int64_t n)
{
    size_t sort_b = 0;
    if (rocprim::radix_sort_pairs(nullptr, sort_b, (unsigned *)nullptr, (unsigned *)nullptr, (int *)nullptr,
                                  (int *)nullptr, (int)n, 0u, 32u) != hipSuccess)
        return 0;
    const size_t a = ((size_t)(n > 0 ? n : 1) * 4 + 255) & ~(size_t)255;
    return 4 * a + sort_b;
}

hipError_t launch_prim_density(const double *drec, const double *sigma, const int32_t *map, int64_t n,
                               const double *prec, int64_t np, double *sbar, int *bad, void *ws, size_t ws_bytes,
                               hipStream_t s)
{
    if (np <= 0 || n <= 0) return hipSuccess;
    const size_t need = prim_density_workspace(n);
    if (!need || !ws || ws_bytes < need) return hipErrorInvalidValue;
    const size_t a = ((size_t)n * 4 + 255) & ~(size_t)255;
    char *w = static_cast<char *>(ws);
    unsigned *kin = reinterpret_cast<unsigned *>(w), *kout = reinterpret_cast<unsigned *>(w + a);
    int *iin = reinterpret_cast<int *>(w + 2 * a), *iout = reinterpret_cast<int *>(w + 3 * a);
    const unsigned gn = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_prim_keys, dim3(gn), dim3(kBlock), 0, s, map, (int)n, (int)np, kin, iin, bad);
    size_t sort_b = need - 4 * a;
    hipError_t e = rocprim::radix_sort_pairs(w + 4 * a, sort_b, kin, kout, iin, iout, (int)n, 0u, 32u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prim_density, dim3((unsigned)((np + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, drec, sigma,
                       kout, iout, (int)n, prec, (int)np, sbar);
    return hipGetLastError();
}

// ------------------------------------------------- several sigma columns
// Weighting fields: K density columns over the same elements and points
// (column k of sigma at sigma + k n).  Each element's copies are summed once
// per point (the closed forms do not depend on sigma) and the K columns take
// their own FP64 sums in the same fixed order as eval_block, so column k's
// results equal a single-column evaluation with that column bit for bit.
// Output (component c, column k) goes to out[c] + k * ostride (out[c] may be
// null: that component is not stored).
template <bool MIXED, int K>
__device__ __forceinline__ void eval_block_multi(const double *__restrict__ drec, const double *__restrict__ sigma,
                                                 int n, int64_t sig_stride, const ImgArgs &img, double near_factor,
                                                 const double *__restrict__ px, const double *__restrict__ py,
                                                 const double *__restrict__ pz, int m, int base_pt, double scale,
                                                 OutCols out)
{
    __shared__ double t_rec[kTileE * R_STRIDE];
    __shared__ double t_sig[kTileE * K];
    const int i = base_pt + threadIdx.x;
    const bool act = i < m;
    const double Px = act ? px[i] : 0.0;
    const double Py = act ? py[i] : 0.0;
    const double Pz = act ? pz[i] : 0.0;
    double aphi[K], aex[K], aey[K], aez[K];
#pragma unroll
    for (int k = 0; k < K; ++k) aphi[k] = aex[k] = aey[k] = aez[k] = 0.0;
    for (int base = 0; base < n; base += kTileE) {
        const int cnt = min(kTileE, n - base);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * R_STRIDE; q += kBlock) t_rec[q] = drec[(size_t)base * R_STRIDE + q];
        for (int q = threadIdx.x; q < cnt * K; q += kBlock) {
            const int pp = q / K, k = q % K;
            t_sig[q] = sigma[(size_t)k * sig_stride + base + pp];
        }
        __syncthreads();
        for (int p = 0; p < cnt; ++p) {
            const Elem e = load_elem(t_rec + p * R_STRIDE);
            if (MIXED && e.kind >= 2 && p + 1 < cnt) {
                // a triangle pair inside this tile, as in eval_block
                const int q1 = e.kind == 2 ? p : p + 1, q2 = e.kind == 2 ? p + 1 : p;
                double sg1[K], sg2[K], c[K][4];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    sg1[k] = uni(t_sig[q1 * K + k]);
                    sg2[k] = uni(t_sig[q2 * K + k]);
                }
                element_pair_copies_mixed<K, false>(load_elem(t_rec + q1 * R_STRIDE),
                                                    load_pair_b(t_rec + q2 * R_STRIDE), sg1, sg2, img, near_factor, Px,
                                                    Py, Pz, c);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    aphi[k] += c[k][0];
                    aex[k] += c[k][1];
                    aey[k] += c[k][2];
                    aez[k] += c[k][3];
                }
                ++p;
                continue;
            }
            if (!MIXED && e.kind >= 2 && p + 1 < cnt) {
                // a triangle pair inside this tile, as in eval_block
                const int q1 = e.kind == 2 ? p : p + 1, q2 = e.kind == 2 ? p + 1 : p;
                double c[2][4];
                element_pair_copies<false>(load_elem(t_rec + q1 * R_STRIDE), load_pair_b(t_rec + q2 * R_STRIDE), img,
                                           Px, Py, Pz, c[q1 - p], c[q2 - p]);
                const double(&c1)[4] = c[0], (&c2)[4] = c[1];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double s1 = uni(t_sig[p * K + k]), s2 = uni(t_sig[(p + 1) * K + k]);
                    aphi[k] = fma(s2, c2[0], fma(s1, c1[0], aphi[k]));
                    aex[k] = fma(s2, c2[1], fma(s1, c1[1], aex[k]));
                    aey[k] = fma(s2, c2[2], fma(s1, c1[2], aey[k]));
                    aez[k] = fma(s2, c2[3], fma(s1, c1[3], aez[k]));
                }
                ++p;
                continue;
            }
            double cp, cx, cy, cz;
            element_copies<MIXED>(e, img, Px, Py, Pz, false, near_factor, cp, cx, cy, cz);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double sg = uni(t_sig[p * K + k]);
                aphi[k] = fma(sg, cp, aphi[k]);
                aex[k] = fma(sg, cx, aex[k]);
                aey[k] = fma(sg, cy, aey[k]);
                aez[k] = fma(sg, cz, aez[k]);
            }
        }
    }
    if (act) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t o = (size_t)k * out.stride + i;
            if (out.c[0]) out.c[0][o] = scale * aphi[k];
            if (out.c[1]) out.c[1][o] = scale * aex[k];
            if (out.c[2]) out.c[2][o] = scale * aey[k];
            if (out.c[3]) out.c[3][o] = scale * aez[k];
        }
    }
}

// outputs of segment `seg`: every stored component moved by seg * seg_stride
__device__ __forceinline__ OutCols seg_out(OutCols o, int seg, int64_t seg_stride)
{
    const size_t so = (size_t)seg * (size_t)seg_stride;
#pragma unroll
    for (int c = 0; c < 4; ++c) o.c[c] = o.c[c] ? o.c[c] + so : nullptr;
    return o;
}

// grid as k_eval_fp64: x over point blocks, y over element segments
template <int K>
__global__ __launch_bounds__(kBlock) void k_eval_multi_fp64(const double *__restrict__ drec,
                                                            const double *__restrict__ sigma, int n,
                                                            int64_t sig_stride, int segsz, ImgArgs img,
                                                            double near_factor, const double *__restrict__ px,
                                                            const double *__restrict__ py,
                                                            const double *__restrict__ pz, int m, double scale,
                                                            OutCols out, int64_t seg_stride)
{
    const int e0 = blockIdx.y * segsz;
    eval_block_multi<false, K>(drec + (size_t)e0 * R_STRIDE, sigma + e0, min(segsz, n - e0), sig_stride, img,
                               near_factor, px, py, pz, m, blockIdx.x * kBlock, scale,
                               seg_out(out, blockIdx.y, seg_stride));
}

// at most 256 VGPRs so that two waves share a SIMD (unbounded, K = 3 and 4
// would take 258 and 266)
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_eval_multi_mixed(
    const double *__restrict__ drec, const double *__restrict__ sigma, int n, int64_t sig_stride, int segsz,
    ImgArgs img, double near_factor, const double *__restrict__ px, const double *__restrict__ py,
    const double *__restrict__ pz, int m, double scale, OutCols out, int64_t seg_stride)
{
    const int e0 = blockIdx.y * segsz;
    eval_block_multi<true, K>(drec + (size_t)e0 * R_STRIDE, sigma + e0, min(segsz, n - e0), sig_stride, img,
                              near_factor, px, py, pz, m, blockIdx.x * kBlock, scale,
                              seg_out(out, blockIdx.y, seg_stride));
}

template <int K>
static void launch_multi_k(const double *drec, const double *sigma, int n, int64_t sig_stride, const SegPlan &sp,
                           const ImgArgs &img, int mixed, double near_factor, const double *px, const double *py,
                           const double *pz, int m, double scale, const OutCols &out, int64_t seg_stride,
                           hipStream_t s)
{
    const dim3 g((unsigned)((m + kBlock - 1) / kBlock), (unsigned)sp.nseg);
    if (mixed)
        hipLaunchKernelGGL(k_eval_multi_mixed<K>, g, dim3(kBlock), 0, s, drec, sigma, n, sig_stride, sp.segsz, img,
                           near_factor, px, py, pz, m, scale, out, seg_stride);
    else
        hipLaunchKernelGGL(k_eval_multi_fp64<K>, g, dim3(kBlock), 0, s, drec, sigma, n, sig_stride, sp.segsz, img,
                           near_factor, px, py, pz, m, scale, out, seg_stride);
}

void launch_eval_multi_seg(const double *drec, const double *sigma, int64_t n, int64_t sig_stride, int ncol,
                           const SegPlan &sp, const ImgArgs &img, int mixed, double near_factor, const double *px,
                           const double *py, const double *pz, int64_t m, double scale, const OutCols &out,
                           int64_t seg_stride, hipStream_t s)
{
    if (m <= 0 || ncol <= 0 || n <= 0) return;
    const int nn = (int)n, mm = (int)m;
    switch (ncol) {
    case 1:
        launch_multi_k<1>(drec, sigma, nn, sig_stride, sp, img, mixed, near_factor, px, py, pz, mm, scale, out,
                          seg_stride, s);
        break;
    case 2:
        launch_multi_k<2>(drec, sigma, nn, sig_stride, sp, img, mixed, near_factor, px, py, pz, mm, scale, out,
                          seg_stride, s);
        break;
    case 3:
        launch_multi_k<3>(drec, sigma, nn, sig_stride, sp, img, mixed, near_factor, px, py, pz, mm, scale, out,
                          seg_stride, s);
        break;
    default:
        launch_multi_k<4>(drec, sigma, nn, sig_stride, sp, img, mixed, near_factor, px, py, pz, mm, scale, out,
                          seg_stride, s);
        break;
    }
}

// Continuous-batching evaluation: workgroup (one wave) b takes work item b --
// up to 64 points of one request against one segment of the elements of one
// resident geometry -- and writes the segment's unscaled partial sums.  The
// per-point arithmetic does not depend on which other items share the launch.
__global__ __launch_bounds__(64) void k_eval_items_fp64(const WorkItem *__restrict__ items,
                                                       const ImgArgs *__restrict__ imgs, double near_factor)
{
    const WorkItem &w = items[blockIdx.x];
    eval_block<false, 64>(w.drec, w.sigma, w.n, imgs[w.geom], near_factor, w.px, w.py, w.pz, w.count, 0, 1.0, w.phi,
                          w.ex, w.ey, w.ez);
}

// two waves per SIMD, as k_eval_mixed
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_eval_items_mixed(
    const WorkItem *__restrict__ items, const ImgArgs *__restrict__ imgs, double near_factor)
{
    const WorkItem &w = items[blockIdx.x];
    eval_block<true, 64>(w.drec, w.sigma, w.n, imgs[w.geom], near_factor, w.px, w.py, w.pz, w.count, 0, 1.0, w.phi,
                         w.ex, w.ey, w.ez);
}

int eval_items_slots(int mixed)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    const hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eval_items_mixed, 64, 0)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eval_items_fp64, 64, 0);
    return (e == hipSuccess && per_cu > 0) ? cus * per_cu : 1;
}

void launch_eval_items(const WorkItem *items, int nitems, const ImgArgs *imgs, int mixed, double near_factor,
                       hipStream_t s)
{
    if (nitems <= 0) return;
    if (mixed)
        hipLaunchKernelGGL(k_eval_items_mixed, dim3(nitems), dim3(64), 0, s, items, imgs, near_factor);
    else
        hipLaunchKernelGGL(k_eval_items_fp64, dim3(nitems), dim3(64), 0, s, items, imgs, near_factor);
}

// Segment partial sums -> results: for column k < ncol and component c,
// out.c[c][k * out.stride + i] = k_e (0 + sum over s = 0 .. nseg-1, in that
// order, of part[s * seg_stride + (4 k + c) m + i]); null components skipped.
__global__ __launch_bounds__(kBlock) void k_reduce_segments(const double *__restrict__ part, int nseg, int ncol,
                                                             int m, int64_t seg_stride, OutCols out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    for (int k = 0; k < ncol; ++k)
        for (int c = 0; c < 4; ++c) {
            if (!out.c[c]) continue;
            const double *p = part + (size_t)(4 * k + c) * m + i;
            double acc = 0.0;
            for (int s = 0; s < nseg; ++s) acc += p[(size_t)s * (size_t)seg_stride];
            out.c[c][(size_t)k * out.stride + i] = kKe * acc;
        }
}

void launch_reduce_segments(const double *part, int nseg, int ncol, int64_t m, int64_t seg_stride,
                            const OutCols &out, hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_reduce_segments, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, part, nseg,
                       ncol, (int)m, seg_stride, out);
}

// ---------------------------------------------------------------- assembly
// Grid: x over blocks of 256 rows, y over blocks of kTileA columns.  Each
// lane writes A[i + j n] for its row i and the block's columns j: the 256
// lanes of a workgroup store 256 consecutive doubles of a column (2 KB).
// The matrix is assembled with the exact closed forms in both precision
// modes: it is a small share of a step's interactions, and far-field
// truncation in its entries would carry into sigma through the solve.
__global__ __launch_bounds__(kBlock) void k_assemble(const double *__restrict__ drec, int n, ImgArgs img,
                                                      const double *__restrict__ cx, const double *__restrict__ cy,
                                                      const double *__restrict__ cz, double *__restrict__ A)
{
    __shared__ double t_rec[kTileA * R_STRIDE];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int j0 = blockIdx.y * kTileA;
    const int cnt = min(kTileA, n - j0);
    for (int k = threadIdx.x; k < cnt * R_STRIDE; k += kBlock) t_rec[k] = drec[(size_t)j0 * R_STRIDE + k];
    __syncthreads();
    if (i >= n) return;
    const double *ri = drec + (size_t)i * R_STRIDE;
    const double Px = cx ? cx[i] : ri[R_CX];
    const double Py = cy ? cy[i] : ri[R_CY];
    const double Pz = cz ? cz[i] : ri[R_CZ];
    const bool diel = ri[R_BC] != 0.0;
    const double nx = ri[R_E3X], ny = ri[R_E3Y], nz = ri[R_E3Z];
    const double jump = ri[R_JUMP];
    for (int p = 0; p < cnt; ++p) {
        const int j = j0 + p;
        const Elem e = load_elem(t_rec + p * R_STRIDE);
        double cp, gx, gy, gz;
        element_copies<false>(e, img, Px, Py, Pz, i == j, 0.0, cp, gx, gy, gz);
        double a = diel ? kKe * (nx * gx + ny * gy + nz * gz) : kKe * cp;
        a += (diel && i == j) ? jump : 0.0;
        A[(size_t)j * n + i] = a;
    }
}

void launch_assemble(const double *drec, int64_t n, const ImgArgs &img, const double *cx, const double *cy,
                     const double *cz, double *A, hipStream_t s)
{
    if (n <= 0) return;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock), (unsigned)((n + kTileA - 1) / kTileA));
    hipLaunchKernelGGL(k_assemble, g, dim3(kBlock), 0, s, drec, (int)n, img, cx, cy, cz, A);
}

}  // namespace nebem
