// line_kernels.hip -- point charges reduced to line charges (the paper's
// Algorithm 3, voxelisation) and the field of uniformly charged segments.
//
// The reduction is deterministic: instead of atomics into voxels, the
// charges are radix-sorted by voxel index (stable, so a voxel's charges keep
// their input order), occupied voxels are found by comparing neighbours,
// numbered by a prefix sum, and each line sums its voxel's charges in order.
// Each occupied voxel gives one segment parallel to z over the voxel's z
// extent, carrying the voxel's total charge uniformly: through the voxel's
// centre in x, y (Algorithm 3's voxel record holds only the total charge
// and the occupancy), or at the |q|-weighted mean x, y of its charges.
//
// Field at the charges themselves (k_line_near): the lines stand in for the
// charges of far voxels only; each charge takes the charges of its own voxel
// and the 26 around it one by one and the lines of every other voxel, so no
// charge sits on or next to a line that contains it.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

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

// line l: the sorted run [start[l], start[l+1]) of one voxel; lkey[l] =
// that voxel's index.  weighted == 0: through the voxel centre; else at the
// |q|-weighted mean x, y, taken relative to the voxel's first charge so that
// the line of a lone charge passes exactly through it (the voxel centre if
// the weights sum to zero).
__global__ __launch_bounds__(kLB) void k_make_lines(const unsigned *__restrict__ key, const int *__restrict__ idx,
                                                    const int *__restrict__ start, int nlines, int nvalid,
                                                    const double *__restrict__ qx, const double *__restrict__ qy,
                                                    const double *__restrict__ q, GridArgs g, int weighted,
                                                    double *__restrict__ lines, unsigned *__restrict__ lkey)
{
    const int l = blockIdx.x * kLB + threadIdx.x;
    if (l >= nlines) return;
    const int s0 = start[l], s1 = (l + 1 < nlines) ? start[l + 1] : nvalid;
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
    const bool wm = weighted && W > 0.0;
    const double x = wm ? x0 + cx / W : g.origin[0] + (i + 0.5) * g.step[0];
    const double y = wm ? y0 + cy / W : g.origin[1] + (j + 0.5) * g.step[1];
    const double z0 = g.origin[2] + k * g.step[2];
    double *o = lines + 7 * (size_t)l;
    o[0] = x;
    o[1] = y;
    o[2] = z0;
    o[3] = x;
    o[4] = y;
    o[5] = z0 + g.step[2];
    o[6] = Q / g.step[2];
    lkey[l] = v;
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
__device__ __forceinline__ void stage_segment(const double *__restrict__ g, double *__restrict__ o)
{
    const double d0 = g[3] - g[0], d1 = g[4] - g[1], d2 = g[5] - g[2];
    const double L = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    // divisions, so that an axis-parallel segment's direction is exact; a
    // point segment carries no charge
    o[0] = g[0];
    o[1] = g[1];
    o[2] = g[2];
    o[3] = L > 0.0 ? d0 / L : 0.0;
    o[4] = L > 0.0 ? d1 / L : 0.0;
    o[5] = L > 0.0 ? d2 / L : 1.0;
    o[6] = L;
    o[7] = L > 0.0 ? g[6] : 0.0;
}

// adds lambda x (potential, field) of one staged segment s at P (unscaled)
__device__ __forceinline__ void segment_add(const double *s, double P0, double P1, double P2, double &ap, double &a0,
                                            double &a1, double &a2)
{
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
        if ((int)threadIdx.x < cnt) stage_segment(lines + 7 * (size_t)(base + threadIdx.x), t + 8 * threadIdx.x);
        __syncthreads();
        for (int l = 0; l < cnt; ++l) segment_add(t + 8 * l, P0, P1, P2, ap, a0, a1, a2);
    }
    if (act) {
        if (phi) phi[i] = kKe * ap;
        if (ex) ex[i] = kKe * a0;
        if (ey) ey[i] = kKe * a1;
        if (ez) ez[i] = kKe * a2;
    }
}

// voxel (i, j, k) of a point, or false outside the grid (as k_voxel_keys)
__device__ __forceinline__ bool voxel_of(double x, double y, double z, const GridArgs &g, int &i, int &j, int &k)
{
    const double u[3] = {floor((x - g.origin[0]) / g.step[0]), floor((y - g.origin[1]) / g.step[1]),
                         floor((z - g.origin[2]) / g.step[2])};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) in = in && u[a] >= 0.0 && u[a] < (double)g.n[a];
    i = in ? (int)u[0] : 0;
    j = in ? (int)u[1] : 0;
    k = in ? (int)u[2] : 0;
    return in;
}

// Field of the lines at the charges themselves, far part: every line except
// those of the charge's own voxel and the 26 around it (a charge outside the
// grid takes every line).  Written (not added) to ex/ey/ez, scaled by k_e.
__global__ __launch_bounds__(kLB) void k_line_field_far(const double *__restrict__ lines,
                                                        const unsigned *__restrict__ lkey, int nl, GridArgs g,
                                                        const double *__restrict__ px, const double *__restrict__ py,
                                                        const double *__restrict__ pz, int m,
                                                        double *__restrict__ ex, double *__restrict__ ey,
                                                        double *__restrict__ ez)
{
    __shared__ double t[kLB * 8];
    __shared__ int tv[kLB * 3];
    const int i = blockIdx.x * kLB + threadIdx.x;
    const bool act = i < m;
    const double P0 = act ? px[i] : 0.0, P1 = act ? py[i] : 0.0, P2 = act ? pz[i] : 0.0;
    int vi, vj, vk;
    const bool in = voxel_of(P0, P1, P2, g, vi, vj, vk);
    double ap = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int base = 0; base < nl; base += kLB) {
        const int cnt = min(kLB, nl - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            stage_segment(lines + 7 * (size_t)(base + threadIdx.x), t + 8 * threadIdx.x);
            const unsigned v = lkey[base + threadIdx.x];
            tv[3 * threadIdx.x] = (int)(v % (unsigned)g.n[0]);
            tv[3 * threadIdx.x + 1] = (int)((v / (unsigned)g.n[0]) % (unsigned)g.n[1]);
            tv[3 * threadIdx.x + 2] = (int)(v / ((unsigned)g.n[0] * (unsigned)g.n[1]));
        }
        __syncthreads();
        for (int l = 0; l < cnt; ++l) {
            const bool near = in && abs(tv[3 * l] - vi) <= 1 && abs(tv[3 * l + 1] - vj) <= 1 &&
                              abs(tv[3 * l + 2] - vk) <= 1;
            if (!near) segment_add(t + 8 * l, P0, P1, P2, ap, a0, a1, a2);
        }
    }
    if (act) {
        ex[i] = kKe * a0;
        ey[i] = kKe * a1;
        ez[i] = kKe * a2;
    }
}

// first l in [0, nl) with lkey[l] == v, or -1 (lkey increasing)
__device__ __forceinline__ int find_line(const unsigned *__restrict__ lkey, int nl, unsigned v)
{
    int lo = 0, hi = nl;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lkey[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < nl && lkey[lo] == v) ? lo : -1;
}

// Near part: one lane per charge inside the grid (sorted position t, charge
// idx[t]); the charges of its own voxel and the 26 around it, each pair in
// FP32 with runs of up to 64 sources summed in FP32 and added to FP64;
// coincident charges (the charge itself included) are skipped.  Added to
// ex/ey/ez, scaled by k_e.
constexpr int kNearRun = 64;
__global__ __launch_bounds__(kLB) void k_line_near(const unsigned *__restrict__ key, const int *__restrict__ idx,
                                                   const int *__restrict__ start, const unsigned *__restrict__ lkey,
                                                   int nl, const int *__restrict__ nvalid_p, GridArgs g,
                                                   const double *__restrict__ qx, const double *__restrict__ qy,
                                                   const double *__restrict__ qz, const double *__restrict__ q,
                                                   double *__restrict__ ex, double *__restrict__ ey,
                                                   double *__restrict__ ez)
{
    const int nvalid = *nvalid_p;
    const int t = blockIdx.x * kLB + threadIdx.x;
    if (t >= nvalid) return;
    const int c = idx[t];
    const double xi = qx[c], yi = qy[c], zi = qz[c];
    const unsigned v = key[t];
    const int vi = (int)(v % (unsigned)g.n[0]);
    const int vj = (int)((v / (unsigned)g.n[0]) % (unsigned)g.n[1]);
    const int vk = (int)(v / ((unsigned)g.n[0] * (unsigned)g.n[1]));
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                const int i = vi + di, j = vj + dj, k = vk + dk;
                if (i < 0 || j < 0 || k < 0 || i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) continue;
                const unsigned w = (unsigned)i + (unsigned)g.n[0] * ((unsigned)j + (unsigned)g.n[1] * (unsigned)k);
                const int l = find_line(lkey, nl, w);
                if (l < 0) continue;
                const int s1 = l + 1 < nl ? start[l + 1] : nvalid;
                for (int r0 = start[l]; r0 < s1; r0 += kNearRun) {
                    const int r1 = min(s1, r0 + kNearRun);
                    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
                    for (int r = r0; r < r1; ++r) {
                        const int c2 = idx[r];
                        const float dx = (float)(xi - qx[c2]);
                        const float dy = (float)(yi - qy[c2]);
                        const float dz = (float)(zi - qz[c2]);
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const float ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                        const float sc = (float)q[c2] * (ir * ir * ir);
                        fx = fmaf(sc, dx, fx);
                        fy = fmaf(sc, dy, fy);
                        fz = fmaf(sc, dz, fz);
                    }
                    ax += (double)fx;
                    ay += (double)fy;
                    az += (double)fz;
                }
            }
    ex[c] += kKe * ax;
    ey[c] += kKe * ay;
    ez[c] += kKe * az;
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

// workspace of one reduction: keys in/out, charge indices in/out, run flags
// (then the lines' voxel keys), run positions, run starts, the count of
// charges inside, sort and scan scratch
bool voxel_layout(int nq, VoxelLayout &L)
{
    size_t sort_b = 0, scan_b = 0;
    if (rocprim::radix_sort_pairs(nullptr, sort_b, (unsigned *)nullptr, (unsigned *)nullptr, (int *)nullptr,
                                  (int *)nullptr, nq, 0u, 32u) != hipSuccess)
        return false;
    if (rocprim::exclusive_scan(nullptr, scan_b, (int *)nullptr, (int *)nullptr, 0, (size_t)nq,
                                rocprim::plus<int>()) != hipSuccess)
        return false;
    const size_t n4 = align256l((size_t)(nq > 0 ? nq : 1) * 4);
    L.kin = 0;
    L.kout = n4;
    L.iin = 2 * n4;
    L.iout = 3 * n4;
    L.flag = 4 * n4;
    L.pos = 5 * n4;
    L.start = 6 * n4;
    L.nvalid = 7 * n4;
    L.sortw = 7 * n4 + 256;
    L.sort_bytes = sort_b;
    L.scanw = L.sortw + align256l(sort_b);
    L.scan_bytes = scan_b;
    L.total = L.scanw + align256l(scan_b);
    return true;
}

size_t voxel_workspace(int nq)
{
    VoxelLayout L;
    return voxel_layout(nq, L) ? L.total : 0;
}

hipError_t voxel_lines(const double *qx, const double *qy, const double *qz, const double *q, int nq,
                       const GridArgs &g, int weighted, double *lines, int64_t max_lines, int64_t *nlines,
                       int64_t *outside, void *ws, size_t ws_bytes, hipStream_t s)
{
    *nlines = 0;
    if (outside) *outside = 0;
    if (nq <= 0) return hipSuccess;
    VoxelLayout L;
    if (!voxel_layout(nq, L) || !ws || ws_bytes < L.total) return hipErrorInvalidValue;
    char *w = static_cast<char *>(ws);
    unsigned *kin = reinterpret_cast<unsigned *>(w + L.kin), *kout = reinterpret_cast<unsigned *>(w + L.kout);
    int *iin = reinterpret_cast<int *>(w + L.iin), *iout = reinterpret_cast<int *>(w + L.iout);
    int *flag = reinterpret_cast<int *>(w + L.flag), *pos = reinterpret_cast<int *>(w + L.pos);
    int *start = reinterpret_cast<int *>(w + L.start), *nvalid = reinterpret_cast<int *>(w + L.nvalid);
    const unsigned gq = (unsigned)((nq + kLB - 1) / kLB);
    int hv[2] = {0, 0};
    hipLaunchKernelGGL(k_voxel_keys, dim3(gq), dim3(kLB), 0, s, qx, qy, qz, nq, g, kin, iin);
    size_t sort_b = L.sort_bytes, scan_b = L.scan_bytes;
    hipError_t e = rocprim::radix_sort_pairs(w + L.sortw, sort_b, kin, kout, iin, iout, nq, 0u, 32u, s);
    if (e == hipSuccess) e = hipMemsetAsync(nvalid, 0, sizeof(int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_run_starts, dim3(gq), dim3(kLB), 0, s, kout, nq, flag, nvalid);
        e = rocprim::exclusive_scan(w + L.scanw, scan_b, flag, pos, 0, (size_t)nq, rocprim::plus<int>(), s);
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
        // the flags are spent: their room takes the lines' voxel keys
        if (hv[0] <= max_lines && hv[0] > 0 && lines)
            hipLaunchKernelGGL(k_make_lines, dim3((unsigned)((hv[0] + kLB - 1) / kLB)), dim3(kLB), 0, s, kout, iout,
                               start, hv[0], hv[1], qx, qy, q, g, weighted, lines,
                               reinterpret_cast<unsigned *>(flag));
        e = hipGetLastError();
    }
    return e;
}

void launch_line_field(const double *lines, int64_t nl, const double *px, const double *py, const double *pz,
                       int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_line_field, dim3((unsigned)((m + kLB - 1) / kLB)), dim3(kLB), 0, s, lines, (int)nl, px, py,
                       pz, (int)m, phi, ex, ey, ez);
}

void launch_line_field_at_charges(const double *lines, int64_t nl, const void *ws, const GridArgs &g,
                                  const double *qx, const double *qy, const double *qz, const double *q, int nq,
                                  double *ex, double *ey, double *ez, hipStream_t s)
{
    if (nq <= 0) return;
    VoxelLayout L;
    if (!voxel_layout(nq, L)) return;
    const char *w = static_cast<const char *>(ws);
    const unsigned *kout = reinterpret_cast<const unsigned *>(w + L.kout);
    const int *iout = reinterpret_cast<const int *>(w + L.iout);
    const int *start = reinterpret_cast<const int *>(w + L.start);
    const int *nvalid = reinterpret_cast<const int *>(w + L.nvalid);
    const unsigned *lkey = reinterpret_cast<const unsigned *>(w + L.flag);
    const unsigned gq = (unsigned)((nq + kLB - 1) / kLB);
    hipLaunchKernelGGL(k_line_field_far, dim3(gq), dim3(kLB), 0, s, lines, lkey, (int)nl, g, qx, qy, qz, nq, ex, ey,
                       ez);
    if (nl > 0)
        hipLaunchKernelGGL(k_line_near, dim3(gq), dim3(kLB), 0, s, kout, iout, start, lkey, (int)nl, nvalid, g, qx, qy,
                           qz, q, ex, ey, ez);
}

}  // namespace nebem
