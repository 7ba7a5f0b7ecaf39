// fastvol_kernels.hip -- FastVolume (the paper's Sec. 3 volume sampling):
// phi and E precomputed once at the nodes of a grid, then trilinear
// interpolation at any number of points.  Two grids: regular (origin, step)
// and graded (a strictly increasing list of node coordinates per axis, so
// that nodes can be dense where the field varies fast -- near electrodes and
// holes -- and sparse in the uniform drift field).
//
// Node values are interleaved, 4 doubles per node (phi, ex, ey, ez), node
// (i, j, k) at 4 (i + nx (j + ny k)): one interpolation gathers 8 corners x
// 32 contiguous bytes (two 16-byte loads each) instead of 32 scattered
// scalars.  The lookup is a gather from an L2/HBM-resident table; per point
// it reads 24 B of coordinates and writes up to 32 B.
#include <hip/hip_runtime.h>

#include <cmath>

#include "nebem_internal.hpp"

namespace nebem {

constexpr int kFB = 256;

// node coordinates, node q = i + nx (j + ny k): origin + i * step with the
// product and the sum each rounded (no FMA), the plain expression's value
__global__ __launch_bounds__(kFB) void k_grid_nodes(GridArgs g, double *__restrict__ px, double *__restrict__ py,
                                                    double *__restrict__ pz)
{
#pragma clang fp contract(off)
    const int64_t q = (int64_t)blockIdx.x * kFB + threadIdx.x;
    const int64_t nn = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (q >= nn) return;
    const int i = (int)(q % g.n[0]);
    const int j = (int)((q / g.n[0]) % g.n[1]);
    const int k = (int)(q / ((int64_t)g.n[0] * g.n[1]));
    px[q] = g.origin[0] + (double)i * g.step[0];
    py[q] = g.origin[1] + (double)j * g.step[1];
    pz[q] = g.origin[2] + (double)k * g.step[2];
}

// values[4 q + c] = src[c][q]
__global__ __launch_bounds__(kFB) void k_interleave4(const double *__restrict__ s0, const double *__restrict__ s1,
                                                     const double *__restrict__ s2, const double *__restrict__ s3,
                                                     int64_t nn, double *__restrict__ values)
{
    const int64_t q = (int64_t)blockIdx.x * kFB + threadIdx.x;
    if (q >= nn) return;
    double2 *v = reinterpret_cast<double2 *>(values + 4 * q);
    v[0] = make_double2(s0[q], s1[q]);
    v[1] = make_double2(s2[q], s3[q]);
}

__device__ __forceinline__ void axis_cell(double x, double o, double inv_step, int n, int &i0, double &f, bool &in)
{
    const double u = (x - o) * inv_step;
    in = in && u >= 0.0 && u <= (double)(n - 1);
    int i = (int)floor(u);
    i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
    i0 = i;
    f = u - (double)i;
}

__global__ __launch_bounds__(kFB) void k_fastvol_interp(GridArgs g, const double *__restrict__ values,
                                                        const double *__restrict__ px, const double *__restrict__ py,
                                                        const double *__restrict__ pz, int m, double *__restrict__ phi,
                                                        double *__restrict__ ex, double *__restrict__ ey,
                                                        double *__restrict__ ez)
{
    const int p = blockIdx.x * kFB + threadIdx.x;
    if (p >= m) return;
    bool in = true;
    int i, j, k;
    double fx, fy, fz;
    axis_cell(px[p], g.origin[0], g.inv_step[0], g.n[0], i, fx, in);
    axis_cell(py[p], g.origin[1], g.inv_step[1], g.n[1], j, fy, in);
    axis_cell(pz[p], g.origin[2], g.inv_step[2], g.n[2], k, fz, in);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t sx = 4, sy = 4 * (int64_t)g.n[0], sz = 4 * (int64_t)g.n[0] * g.n[1];
    const double2 *base = reinterpret_cast<const double2 *>(values + i * sx + j * sy + k * sz);
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                const double w = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
                const double2 *c = base + (di * sx + dj * sy + dk * sz) / 2;
                const double2 a = c[0], b = c[1];
                acc[0] = fma(w, a.x, acc[0]);
                acc[1] = fma(w, a.y, acc[1]);
                acc[2] = fma(w, b.x, acc[2]);
                acc[3] = fma(w, b.y, acc[3]);
            }
    const double nan = __builtin_nan("");
    if (phi) phi[p] = in ? acc[0] : nan;
    if (ex) ex[p] = in ? acc[1] : nan;
    if (ey) ey[p] = in ? acc[2] : nan;
    if (ez) ez[p] = in ? acc[3] : nan;
}

// ------------------------------------------------------------ graded grids
__global__ __launch_bounds__(kFB) void k_axes_nodes(AxesArgs g, double *__restrict__ px, double *__restrict__ py,
                                                    double *__restrict__ pz)
{
    const int64_t q = (int64_t)blockIdx.x * kFB + threadIdx.x;
    const int64_t nn = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (q >= nn) return;
    const int i = (int)(q % g.n[0]);
    const int j = (int)((q / g.n[0]) % g.n[1]);
    const int k = (int)(q / ((int64_t)g.n[0] * g.n[1]));
    px[q] = g.ax[0][i];
    py[q] = g.ax[1][j];
    pz[q] = g.ax[2][k];
}

// bad[0] = 1 if any axis is not strictly increasing or not finite (bad
// cleared by the caller)
__global__ __launch_bounds__(kFB) void k_axes_check(AxesArgs g, int *__restrict__ bad)
{
    const int t = blockIdx.x * kFB + threadIdx.x;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (t >= g.n[a]) continue;
        const double v = g.ax[a][t];
        const bool ok = isfinite(v) && (t == 0 || g.ax[a][t - 1] < v);
        if (!ok) bad[0] = 1;
    }
}

// cell of x on a strictly increasing axis a[0..n-1]: the largest i <= n-2
// with a[i] <= x (0 below the first node), fraction f = (x - a[i]) /
// (a[i+1] - a[i]); `in` cleared outside [a[0], a[n-1]].  The search reads
// only a[0..n-1], whatever the values.
__device__ __forceinline__ void axis_cell_graded(double x, const double *__restrict__ a, int n, int &i0, double &f,
                                                 bool &in)
{
    in = in && x >= a[0] && x <= a[n - 1];
    int lo = 0, hi = n - 2;  // answer in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    i0 = lo;
    f = (x - a[lo]) / (a[lo + 1] - a[lo]);
}

__global__ __launch_bounds__(kFB) void k_fastvol_interp_axes(AxesArgs g, const double *__restrict__ values,
                                                             const double *__restrict__ px,
                                                             const double *__restrict__ py,
                                                             const double *__restrict__ pz, int m,
                                                             double *__restrict__ phi, double *__restrict__ ex,
                                                             double *__restrict__ ey, double *__restrict__ ez)
{
    const int p = blockIdx.x * kFB + threadIdx.x;
    if (p >= m) return;
    bool in = true;
    int i, j, k;
    double fx, fy, fz;
    axis_cell_graded(px[p], g.ax[0], g.n[0], i, fx, in);
    axis_cell_graded(py[p], g.ax[1], g.n[1], j, fy, in);
    axis_cell_graded(pz[p], g.ax[2], g.n[2], k, fz, in);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t sx = 4, sy = 4 * (int64_t)g.n[0], sz = 4 * (int64_t)g.n[0] * g.n[1];
    const double2 *base = reinterpret_cast<const double2 *>(values + i * sx + j * sy + k * sz);
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                const double w = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
                const double2 *c = base + (di * sx + dj * sy + dk * sz) / 2;
                const double2 a = c[0], b = c[1];
                acc[0] = fma(w, a.x, acc[0]);
                acc[1] = fma(w, a.y, acc[1]);
                acc[2] = fma(w, b.x, acc[2]);
                acc[3] = fma(w, b.y, acc[3]);
            }
    const double nan = __builtin_nan("");
    if (phi) phi[p] = in ? acc[0] : nan;
    if (ex) ex[p] = in ? acc[1] : nan;
    if (ey) ey[p] = in ? acc[2] : nan;
    if (ez) ez[p] = in ? acc[3] : nan;
}

void launch_axes_nodes(const AxesArgs &g, double *px, double *py, double *pz, hipStream_t s)
{
    const int64_t nn = (int64_t)g.n[0] * g.n[1] * g.n[2];
    hipLaunchKernelGGL(k_axes_nodes, dim3((unsigned)((nn + kFB - 1) / kFB)), dim3(kFB), 0, s, g, px, py, pz);
}

void launch_axes_check(const AxesArgs &g, int *bad, hipStream_t s)
{
    const int nmax = g.n[0] > g.n[1] ? (g.n[0] > g.n[2] ? g.n[0] : g.n[2]) : (g.n[1] > g.n[2] ? g.n[1] : g.n[2]);
    hipLaunchKernelGGL(k_axes_check, dim3((unsigned)((nmax + kFB - 1) / kFB)), dim3(kFB), 0, s, g, bad);
}

void launch_fastvol_interp_axes(const AxesArgs &g, const double *values, const double *px, const double *py,
                                const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                                hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_fastvol_interp_axes, dim3((unsigned)((m + kFB - 1) / kFB)), dim3(kFB), 0, s, g, values, px,
                       py, pz, (int)m, phi, ex, ey, ez);
}

void launch_grid_nodes(const GridArgs &g, double *px, double *py, double *pz, hipStream_t s)
{
    const int64_t nn = (int64_t)g.n[0] * g.n[1] * g.n[2];
    hipLaunchKernelGGL(k_grid_nodes, dim3((unsigned)((nn + kFB - 1) / kFB)), dim3(kFB), 0, s, g, px, py, pz);
}

void launch_interleave4(const double *s0, const double *s1, const double *s2, const double *s3, int64_t nn,
                        double *values, hipStream_t s)
{
    hipLaunchKernelGGL(k_interleave4, dim3((unsigned)((nn + kFB - 1) / kFB)), dim3(kFB), 0, s, s0, s1, s2, s3, nn,
                       values);
}

void launch_fastvol_interp(const GridArgs &g, const double *values, const double *px, const double *py,
                           const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                           hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_fastvol_interp, dim3((unsigned)((m + kFB - 1) / kFB)), dim3(kFB), 0, s, g, values, px, py,
                       pz, (int)m, phi, ex, ey, ez);
}

}  // namespace nebem
