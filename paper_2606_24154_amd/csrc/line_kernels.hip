// line_kernels.hip -- point charges reduced to line charges (the paper's
// Algorithm 3, voxelisation) and the field of uniformly charged segments.
//
// The reduction is deterministic: instead of atomics into voxels, the
// charges are radix-sorted by voxel index (stable, so a voxel's charges keep
// their input order), occupied voxels are found by comparing neighbours,
// numbered by a prefix sum, and each line sums its voxel's charges in order.
// Each occupied voxel gives one segment parallel to z over the voxel's z
// extent, at the |q|-weighted mean x, y of its charges (the voxel centre if
// that weight is zero), carrying the voxel's total charge uniformly.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "fastmath_fp64.hpp"
#include "nebem_internal.hpp"

namespace nebem {

constexpr int kLB = 256;
constexpr unsigned kOutside = 0xffffffffu;

__global__ __launch_bounds__(kLB) void k_voxel_keys(const double *__restrict__ qx, const double *__restrict__ qy,
                                                    const double *__restrict__ qz, int nq, GridArgs g,
                                                    unsigned *__restrict__ key, int *__restrict__ idx)
{
    const int i = blockIdx.x * kLB + threadIdx.x;
    if (i >= nq) return;
    const double x[3] = {qx[i], qy[i], qz[i]};
    long long v[3];
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = floor((x[a] - g.origin[a]) / g.step[a]);
        in = in && u >= 0.0 && u < (double)g.n[a];
        v[a] = in ? (long long)u : 0;
    }
    key[i] = in ? (unsigned)(v[0] + (long long)g.n[0] * (v[1] + (long long)g.n[1] * v[2])) : kOutside;
    idx[i] = i;
}

// flag[i] = 1 where an occupied voxel's run starts; nvalid = charges inside
__global__ __launch_bounds__(kLB) void k_run_starts(const unsigned *__restrict__ key, int nq, int *__restrict__ flag,
                                                    int *__restrict__ nvalid)
{
    const int i = blockIdx.x * kLB + threadIdx.x;
    if (i >= nq) return;
    const unsigned k = key[i];
    flag[i] = (k != kOutside && (i == 0 || key[i - 1] != k)) ? 1 : 0;
    if (k != kOutside && (i == nq - 1 || key[i + 1] == kOutside)) *nvalid = i + 1;
}

__global__ __launch_bounds__(kLB) void k_run_index(const int *__restrict__ flag, const int *__restrict__ pos, int nq,
                                                   int *__restrict__ start)
{
    const int i = blockIdx.x * kLB + threadIdx.x;
    if (i >= nq) return;
    if (flag[i]) start[pos[i]] = i;
}

__global__ __launch_bounds__(kLB) void k_make_lines(const unsigned *__restrict__ key, const int *__restrict__ idx,
                                                    const int *__restrict__ start, int nlines, int nvalid,
                                                    const double *__restrict__ qx, const double *__restrict__ qy,
                                                    const double *__restrict__ q, GridArgs g,
                                                    double *__restrict__ lines)
{
    const int l = blockIdx.x * kLB + threadIdx.x;
    if (l >= nlines) return;
    const int s0 = start[l], s1 = (l + 1 < nlines) ? start[l + 1] : nvalid;
    // weighted mean taken relative to the voxel's first charge, so that the
    // line of a lone charge passes exactly through it
    const double x0 = qx[idx[s0]], y0 = qy[idx[s0]];
    double Q = 0.0, W = 0.0, cx = 0.0, cy = 0.0;
    for (int s = s0; s < s1; ++s) {
        const int c = idx[s];
        const double qc = q[c], w = fabs(qc);
        Q += qc;
        W += w;
        cx += w * (qx[c] - x0);
        cy += w * (qy[c] - y0);
    }
    const unsigned v = key[s0];
    const int i = (int)(v % (unsigned)g.n[0]);
    const int j = (int)((v / (unsigned)g.n[0]) % (unsigned)g.n[1]);
    const int k = (int)(v / ((unsigned)g.n[0] * (unsigned)g.n[1]));
    const double x = W > 0.0 ? x0 + cx / W : g.origin[0] + (i + 0.5) * g.step[0];
    const double y = W > 0.0 ? y0 + cy / W : g.origin[1] + (j + 0.5) * g.step[1];
    const double z0 = g.origin[2] + k * g.step[2];
    double *o = lines + 7 * (size_t)l;
    o[0] = x;
    o[1] = y;
    o[2] = z0;
    o[3] = x;
    o[4] = y;
    o[5] = z0 + g.step[2];
    o[6] = Q / g.step[2];
}

// 1/sqrt(x), x > 0: hardware estimate and two Newton steps
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = fma(y, fma(-hx * y, y, 0.5), y);
    return fma(y, fma(-hx * y, y, 0.5), y);
}

// phi, E of nl segments (7 doubles each: a, b, lambda) at m points, one lane
// per point; k_e applied at the end.  Each tile of segments is staged in LDS
// as (a, unit direction t, length L, lambda), computed once per workgroup.
//
// With s_A = (a - P).t, s_B = s_A + L, rho the distance of P from the line
// and r_A, r_B its distances from the ends (r^2 = rho^2 + s^2), every
// quantity is formed without cancellation:
//   r_B - r_A = L (s_A + s_B)/(r_A + r_B);
//   phi/(k_e lambda) = ln((r_B + s_B)/(r_A + s_A)) = ln(1 + F/D), with
//     F = L (r_A + r_B + |s_A + s_B|)/(r_A + r_B) and D = r_A + s_A if
//     s_A + s_B >= 0, else (mirrored) D = r_B - s_B; a D of the form r + s
//     with s < 0 taken as rho^2/(r - s);
//   1/r_B - 1/r_A = -L (s_A + s_B)/((r_A + r_B) r_A r_B)  (along t);
//   (s_B/r_B - s_A/r_A)/rho^2 (across, along P - foot) as
//     L (s_A + s_B)/((s_B r_A + s_A r_B) r_A r_B) when P is level with or
//     beyond an end (s_A s_B >= 0).
// A point on a segment gets infinite phi and the principal value 0 for the
// field across it; at an end the results are not finite.
__global__ __launch_bounds__(kLB) void k_line_field(const double *__restrict__ lines, int nl,
                                                    const double *__restrict__ px, const double *__restrict__ py,
                                                    const double *__restrict__ pz, int m, double *__restrict__ phi,
                                                    double *__restrict__ ex, double *__restrict__ ey,
                                                    double *__restrict__ ez)
{
    __shared__ double t[kLB * 8];
    const int i = blockIdx.x * kLB + threadIdx.x;
    const bool act = i < m;
    const double P0 = act ? px[i] : 0.0, P1 = act ? py[i] : 0.0, P2 = act ? pz[i] : 0.0;
    double ap = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int base = 0; base < nl; base += kLB) {
        const int cnt = min(kLB, nl - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const double *g = lines + 7 * (size_t)(base + threadIdx.x);
            const double d0 = g[3] - g[0], d1 = g[4] - g[1], d2 = g[5] - g[2];
            const double L = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            // divisions, so that an axis-parallel segment's direction is
            // exact; a point segment carries no charge
            double *o = t + 8 * threadIdx.x;
            o[0] = g[0];
            o[1] = g[1];
            o[2] = g[2];
            o[3] = L > 0.0 ? d0 / L : 0.0;
            o[4] = L > 0.0 ? d1 / L : 0.0;
            o[5] = L > 0.0 ? d2 / L : 1.0;
            o[6] = L;
            o[7] = L > 0.0 ? g[6] : 0.0;
        }
        __syncthreads();
        for (int l = 0; l < cnt; ++l) {
            const double *s = t + 8 * l;
            const double q0 = P0 - s[0], q1 = P1 - s[1], q2 = P2 - s[2];
            const double t0 = s[3], t1 = s[4], t2 = s[5], L = s[6], lam = s[7];
            const double along = fma(q0, t0, fma(q1, t1, q2 * t2));
            const double p0 = fma(-along, t0, q0), p1 = fma(-along, t1, q1), p2 = fma(-along, t2, q2);
            const double rho2 = fma(p0, p0, fma(p1, p1, p2 * p2));
            const double sA = -along, sB = L - along;
            const double rA2 = fma(sA, sA, rho2), rB2 = fma(sB, sB, rho2);
            const double irA = rsq64(rA2), irB = rsq64(rB2);
            const double rA = rA2 * irA, rB = rB2 * irB;
            const double rs = rA + rB, ss = sA + sB;
            // potential
            const bool formA = ss >= 0.0;  // D built on end A, else mirrored onto end B
            const double u = formA ? sA : -sB, v = formA ? rA : rB;
            const bool outside = u >= 0.0;  // level with or beyond an end: s_A s_B >= 0
            const double F = L * (rs + fabs(ss));
            const double nn = outside ? F : F * (v - u);
            const double dd = rs * (outside ? v + u : rho2);
            const double lg = dd > 0.0 ? log1p_ratio(nn, dd) : __builtin_inf();
            // field: one reciprocal serves 1/(r_A + r_B) and the across factor
            const double c = L * ss * irA * irB;
            double gden = outside ? fma(sB, rA, sA * rB) : rho2;
            const bool gok = gden != 0.0;
            gden = gok ? gden : 1.0;
            const double R = rcp64(gden * rs);
            const double gnum = outside ? c : fma(sB, irB, -(sA * irA));
            const double gp = gok ? gnum * (rs * R) : 0.0;
            const double gt = -c * (gden * R);
            ap = fma(lam, lg, ap);
            a0 = fma(lam, fma(gp, p0, gt * t0), a0);
            a1 = fma(lam, fma(gp, p1, gt * t1), a1);
            a2 = fma(lam, fma(gp, p2, gt * t2), a2);
        }
    }
    if (act) {
        if (phi) phi[i] = kKe * ap;
        if (ex) ex[i] = kKe * a0;
        if (ey) ey[i] = kKe * a1;
        if (ez) ez[i] = kKe * a2;
    }
}

// collocation points (element centroids) as three arrays
__global__ __launch_bounds__(kLB) void k_centroids(const double *__restrict__ drec, int n, double *__restrict__ cx,
                                                   double *__restrict__ cy, double *__restrict__ cz)
{
    const int i = blockIdx.x * kLB + threadIdx.x;
    if (i >= n) return;
    const double *r = drec + (size_t)i * R_STRIDE;
    cx[i] = r[R_CX];
    cy[i] = r[R_CY];
    cz[i] = r[R_CZ];
}

// b_i = b0_i - phi_i on conductor rows, b0_i - n_i . E_i on interface rows
__global__ __launch_bounds__(kLB) void k_line_rhs_finish(const double *__restrict__ drec, int n,
                                                         const double *__restrict__ f, const double *__restrict__ b0,
                                                         double *__restrict__ b)
{
    const int i = blockIdx.x * kLB + threadIdx.x;
    if (i >= n) return;
    const double *r = drec + (size_t)i * R_STRIDE;
    const double *phi = f, *ex = f + n, *ey = f + 2 * (size_t)n, *ez = f + 3 * (size_t)n;
    const double en = fma(r[R_E3X], ex[i], fma(r[R_E3Y], ey[i], r[R_E3Z] * ez[i]));
    b[i] = b0[i] - (r[R_BC] != 0.0 ? en : phi[i]);
}

void launch_line_rhs(const double *drec, int64_t n, const double *lines, int64_t nl, const double *b0, double *work,
                     double *b, hipStream_t s)
{
    if (n <= 0) return;
    const unsigned g = (unsigned)((n + kLB - 1) / kLB);
    double *c = work, *f = work + 3 * (size_t)n;
    hipLaunchKernelGGL(k_centroids, dim3(g), dim3(kLB), 0, s, drec, (int)n, c, c + n, c + 2 * n);
    launch_line_field(lines, nl, c, c + n, c + 2 * n, n, f, f + n, f + 2 * n, f + 3 * n, s);
    hipLaunchKernelGGL(k_line_rhs_finish, dim3(g), dim3(kLB), 0, s, drec, (int)n, f, b0, b);
}

static size_t align256l(size_t b) { return (b + 255) & ~(size_t)255; }

// workspace: keys in/out, idx in/out, flags, positions, starts, nvalid, cub scratch
hipError_t voxel_lines(const double *qx, const double *qy, const double *qz, const double *q, int nq,
                       const GridArgs &g, double *lines, int64_t max_lines, int64_t *nlines, int64_t *outside,
                       hipStream_t s)
{
    *nlines = 0;
    if (outside) *outside = 0;
    if (nq <= 0) return hipSuccess;
    size_t sort_b = 0, scan_b = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_b, (unsigned *)nullptr, (unsigned *)nullptr,
                                                      (int *)nullptr, (int *)nullptr, nq, 0, 32, s);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_b, (int *)nullptr, (int *)nullptr, nq, s);
    if (e != hipSuccess) return e;
    const size_t n4 = align256l((size_t)nq * 4);
    const size_t total = 7 * n4 + 256 + align256l(sort_b) + align256l(scan_b);
    void *ws = nullptr;
    if ((e = hipMallocAsync(&ws, total, s)) != hipSuccess) return e;
    char *w = static_cast<char *>(ws);
    unsigned *kin = reinterpret_cast<unsigned *>(w), *kout = reinterpret_cast<unsigned *>(w + n4);
    int *iin = reinterpret_cast<int *>(w + 2 * n4), *iout = reinterpret_cast<int *>(w + 3 * n4);
    int *flag = reinterpret_cast<int *>(w + 4 * n4), *pos = reinterpret_cast<int *>(w + 5 * n4);
    int *start = reinterpret_cast<int *>(w + 6 * n4), *nvalid = reinterpret_cast<int *>(w + 7 * n4);
    void *sortw = w + 7 * n4 + 256, *scanw = w + 7 * n4 + 256 + align256l(sort_b);
    const unsigned gq = (unsigned)((nq + kLB - 1) / kLB);
    int hv[2] = {0, 0};
    hipLaunchKernelGGL(k_voxel_keys, dim3(gq), dim3(kLB), 0, s, qx, qy, qz, nq, g, kin, iin);
    e = hipcub::DeviceRadixSort::SortPairs(sortw, sort_b, kin, kout, iin, iout, nq, 0, 32, s);
    if (e == hipSuccess) e = hipMemsetAsync(nvalid, 0, sizeof(int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_run_starts, dim3(gq), dim3(kLB), 0, s, kout, nq, flag, nvalid);
        e = hipcub::DeviceScan::ExclusiveSum(scanw, scan_b, flag, pos, nq, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_run_index, dim3(gq), dim3(kLB), 0, s, flag, pos, nq, start);
        // lines = pos[nq-1] + flag[nq-1]; nvalid from the device
        int last[2];
        e = hipMemcpyAsync(&last[0], pos + nq - 1, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&last[1], flag + nq - 1, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hv[1], nvalid, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        hv[0] = last[0] + last[1];
    }
    if (e == hipSuccess) {
        *nlines = hv[0];
        if (outside) *outside = nq - hv[1];
        if (hv[0] <= max_lines && hv[0] > 0 && lines)
            hipLaunchKernelGGL(k_make_lines, dim3((unsigned)((hv[0] + kLB - 1) / kLB)), dim3(kLB), 0, s, kout, iout,
                               start, hv[0], hv[1], qx, qy, q, g, lines);
        e = hipGetLastError();
    }
    hipError_t e2 = hipFreeAsync(ws, s);
    return e != hipSuccess ? e : e2;
}

void launch_line_field(const double *lines, int64_t nl, const double *px, const double *py, const double *pz,
                       int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_line_field, dim3((unsigned)((m + kLB - 1) / kLB)), dim3(kLB), 0, s, lines, (int)nl, px, py,
                       pz, (int)m, phi, ex, ey, ez);
}

}  // namespace nebem
