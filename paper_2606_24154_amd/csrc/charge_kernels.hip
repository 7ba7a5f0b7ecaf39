// charge_kernels.hip -- point-charge sums of the dynamic space-charge step
// (paper Sec. 4.2, Algorithm 2: each field point sums q_i/r over the known
// charges; here generalised to the field, to every charge as a target, and to
// the right-hand side of the collocation system) and the explicit-Euler move
// of Sec. 4.3 / Algorithm 4's time step.
//
// Algorithm 2 spreads the sources of ONE field point over a whole grid and
// reduces with shared memory plus one atomic per block.  With a million
// targets there is parallelism enough in the targets themselves: one lane owns
// one target, source positions stream through LDS in tiles shared by the 256
// lanes of a workgroup, and every target's sum has a fixed order -- no atomics,
// run-to-run identical results.
//
// Precision (pair sums): the position difference is formed in FP64 and the
// pair term in FP32; each run of 64 sources is summed in FP32 and then added
// to FP64 accumulators.
#include <hip/hip_runtime.h>

#include "charge_internal.hpp"
#include "nebem_internal.hpp"

namespace nebem {

constexpr int kCB = 256;   // lanes per workgroup = sources per LDS tile
constexpr int kRun = 64;   // sources per FP32 partial sum

// E at every charge from all other charges (added to ex/ey/ez, scaled by k_e)
__global__ __launch_bounds__(kCB) void k_coulomb_self(const double *__restrict__ qx, const double *__restrict__ qy,
                                                      const double *__restrict__ qz, const double *__restrict__ q,
                                                      int nq, double *__restrict__ ex, double *__restrict__ ey,
                                                      double *__restrict__ ez)
{
    __shared__ double sx[kCB], sy[kCB], sz[kCB];
    __shared__ float sq[kCB];
    const int i = blockIdx.x * kCB + threadIdx.x;
    const bool act = i < nq;
    const double xi = act ? qx[i] : 0.0, yi = act ? qy[i] : 0.0, zi = act ? qz[i] : 0.0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int base = 0; base < nq; base += kCB) {
        __syncthreads();
        const int j = base + threadIdx.x;
        if (j < nq) {
            sx[threadIdx.x] = qx[j];
            sy[threadIdx.x] = qy[j];
            sz[threadIdx.x] = qz[j];
            sq[threadIdx.x] = (float)q[j];
        } else {  // padding: zero charge
            sx[threadIdx.x] = 0.0;
            sy[threadIdx.x] = 0.0;
            sz[threadIdx.x] = 0.0;
            sq[threadIdx.x] = 0.0f;
        }
        __syncthreads();
#pragma unroll 1
        for (int r0 = 0; r0 < kCB; r0 += kRun) {
            float fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll 8
            for (int k = r0; k < r0 + kRun; ++k) {
                const float dx = (float)(xi - sx[k]);
                const float dy = (float)(yi - sy[k]);
                const float dz = (float)(zi - sz[k]);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                // the target itself and coincident charges contribute nothing
                const float ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                const float s = sq[k] * (ir * ir * ir);
                fx = fmaf(s, dx, fx);
                fy = fmaf(s, dy, fy);
                fz = fmaf(s, dz, fz);
            }
            ax += (double)fx;
            ay += (double)fy;
            az += (double)fz;
        }
    }
    if (act) {
        ex[i] += kKe * ax;
        ey[i] += kKe * ay;
        ez[i] += kKe * az;
    }
}

// Right-hand side with the known charges (RHVector with the charges' share,
// Sec. 4.1): partial sums over source chunk blockIdx.y for every collocation
// row i -- potential for conductor rows, n_i . E for interface rows.
// part[(size_t)blockIdx.y * n + i]
__global__ __launch_bounds__(kCB) void k_charge_rhs_part(const double *__restrict__ drec, int n,
                                                         const double *__restrict__ qx,
                                                         const double *__restrict__ qy,
                                                         const double *__restrict__ qz,
                                                         const double *__restrict__ q, int nq, int chunk,
                                                         double *__restrict__ part)
{
    __shared__ double sx[kCB], sy[kCB], sz[kCB];
    __shared__ float sq[kCB];
    const int i = blockIdx.x * kCB + threadIdx.x;
    const bool act = i < n;
    const double *ri = drec + (size_t)(act ? i : 0) * R_STRIDE;
    const double xi = ri[R_CX], yi = ri[R_CY], zi = ri[R_CZ];
    const bool diel = ri[R_BC] != 0.0;
    const double nx = ri[R_E3X], ny = ri[R_E3Y], nz = ri[R_E3Z];
    const int j0 = blockIdx.y * chunk, j1 = min(nq, j0 + chunk);
    double acc = 0.0;
    for (int base = j0; base < j1; base += kCB) {
        __syncthreads();
        const int j = base + threadIdx.x;
        const bool ok = j < j1;
        sx[threadIdx.x] = ok ? qx[j] : 0.0;
        sy[threadIdx.x] = ok ? qy[j] : 0.0;
        sz[threadIdx.x] = ok ? qz[j] : 0.0;
        sq[threadIdx.x] = ok ? (float)q[j] : 0.0f;
        __syncthreads();
        float fa = 0.0f;
#pragma unroll 8
        for (int k = 0; k < kCB; ++k) {
            const float dx = (float)(xi - sx[k]);
            const float dy = (float)(yi - sy[k]);
            const float dz = (float)(zi - sz[k]);
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
            // potential: q/r ; normal field: q (n . d)/r^3
            const float nd = diel ? fmaf((float)nx, dx, fmaf((float)ny, dy, (float)nz * dz)) * (ir * ir) : 1.0f;
            fa = fmaf(sq[k] * ir, nd, fa);
            if ((k & (kRun - 1)) == kRun - 1) {
                acc += (double)fa;
                fa = 0.0f;
            }
        }
    }
    if (act) part[(size_t)blockIdx.y * n + i] = acc;
}

// b_i = b0_i - k_e sum_c part[c][i]
__global__ __launch_bounds__(kCB) void k_charge_rhs_finish(const double *__restrict__ part, int n, int nchunk,
                                                           const double *__restrict__ b0, double *__restrict__ b)
{
    const int i = blockIdx.x * kCB + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * n + i];
    b[i] = b0[i] - kKe * s;
}

// x += sign(q) mobility E dt
__global__ __launch_bounds__(kCB) void k_euler(double *__restrict__ qx, double *__restrict__ qy,
                                               double *__restrict__ qz, const double *__restrict__ q,
                                               const double *__restrict__ ex, const double *__restrict__ ey,
                                               const double *__restrict__ ez, int nq, double mu_dt)
{
    const int i = blockIdx.x * kCB + threadIdx.x;
    if (i >= nq) return;
    const double sg = q[i] > 0.0 ? mu_dt : (q[i] < 0.0 ? -mu_dt : 0.0);
    qx[i] = fma(sg, ex[i], qx[i]);
    qy[i] = fma(sg, ey[i], qy[i]);
    qz[i] = fma(sg, ez[i], qz[i]);
}

// b0_i = V_i on conductors, 0 on dielectric interfaces
__global__ __launch_bounds__(kCB) void k_boundary_values(const int *__restrict__ bc, const double *__restrict__ value,
                                                         int n, double *__restrict__ b0)
{
    const int i = blockIdx.x * kCB + threadIdx.x;
    if (i < n) b0[i] = bc[i] == 0 ? (value ? value[i] : 0.0) : 0.0;
}

static inline unsigned blocks(int64_t n) { return (unsigned)((n + kCB - 1) / kCB); }

void launch_coulomb_self(const double *qx, const double *qy, const double *qz, const double *q, int64_t nq, double *ex,
                         double *ey, double *ez, hipStream_t s)
{
    if (nq <= 0) return;
    hipLaunchKernelGGL(k_coulomb_self, dim3(blocks(nq)), dim3(kCB), 0, s, qx, qy, qz, q, (int)nq, ex, ey, ez);
}

int charge_rhs_chunks(int64_t n, int64_t nq)
{
    // aim for >= 2048 workgroups over (rows x source chunks), chunks of >= 4096 sources
    const int64_t rowblocks = (n + kCB - 1) / kCB;
    int64_t want = (2048 + rowblocks - 1) / rowblocks;
    const int64_t maxc = (nq + 4095) / 4096;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    return (int)want;
}

void launch_charge_rhs(const double *drec, int64_t n, const double *qx, const double *qy, const double *qz,
                       const double *q, int64_t nq, const double *b0, double *part, int nchunk, double *b,
                       hipStream_t s)
{
    const int chunk = (int)((nq + nchunk - 1) / nchunk);
    if (nq > 0)
        hipLaunchKernelGGL(k_charge_rhs_part, dim3(blocks(n), nchunk), dim3(kCB), 0, s, drec, (int)n, qx, qy, qz, q,
                           (int)nq, chunk, part);
    hipLaunchKernelGGL(k_charge_rhs_finish, dim3(blocks(n)), dim3(kCB), 0, s, part, (int)n, nq > 0 ? nchunk : 0,
                       b0, b);
}

void launch_euler(double *qx, double *qy, double *qz, const double *q, const double *ex, const double *ey,
                  const double *ez, int64_t nq, double mu_dt, hipStream_t s)
{
    if (nq <= 0) return;
    hipLaunchKernelGGL(k_euler, dim3(blocks(nq)), dim3(kCB), 0, s, qx, qy, qz, q, ex, ey, ez, (int)nq, mu_dt);
}

void launch_boundary_values(const int *bc, const double *value, int64_t n, double *b0, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_boundary_values, dim3(blocks(n)), dim3(kCB), 0, s, bc, value, (int)n, b0);
}

}  // namespace nebem
