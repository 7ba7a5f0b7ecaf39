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
// Pair sums at the charges (k_coulomb_sorted): the charges are first put in
// Morton order of their bounding box, so that every 64 consecutive charges
// -- a wave of targets, a run of sources -- sit in a small box (the boxes of
// all 64-charge runs are computed once per step).  Each source is staged as
// its FP32 offset in micrometres from the centre of its run's box (and as
// its FP64 position).  For a wave and a run whose boxes are at least the
// run's diagonal apart (far), every target first takes its own FP32 offset
// from that centre (once per run, not per pair), and a pair costs 3 FP32
// subtractions, 3 FMAs for r^2 (seeded with 1e-24 um^2, far below any
// resolvable distance, which keeps 1/r^3 finite), one reciprocal square
// root, 2 multiplications and 3 FMAs: 12 VALU instructions.  The source
// offset is at most half a diagonal and the target offset at most the pair
// distance d plus half a diagonal, so their rounding leaves the difference
// within ~1.2e-7 d.  Nearer runs (the wave's own and its spatial
// neighbours: ~8 % of the pairs for a 10^6-charge cloud, against 57 % when
// the test was made per 256 charges) take the difference in FP64 and round
// it once, so close pairs -- whose terms can dominate a charge's field --
// keep the FP32 pair term's own accuracy.  Runs of 64 sources are summed in
// FP32 (eight interleaved sums of 8 in the far runs, where Morton-adjacent
// terms add coherently) and then added to FP64 accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "charge_internal.hpp"
#include "nebem_internal.hpp"

namespace nebem {

constexpr int kCB = 256;   // lanes per workgroup = sources per LDS tile
constexpr int kRun = 64;   // charges per box: a wave of targets, a run of sources

static inline unsigned blocks(int64_t n) { return (unsigned)((n + kCB - 1) / kCB); }
static inline unsigned runs(int64_t n) { return (unsigned)((n + kRun - 1) / kRun); }

constexpr double kUm = 1e6;          // metres -> micrometres for the FP32 offsets
constexpr float kSeedR2 = 1e-24f;    // um^2, keeps 1/r^3 finite at r = 0

// box[6 t .. 6 t + 5] = (min x, y, z, max x, y, z) of sorted charges
// [64 t, 64 t + 64); one 64-lane workgroup per box
__global__ __launch_bounds__(kRun) void k_tile_boxes(const double *__restrict__ sx, const double *__restrict__ sy,
                                                     const double *__restrict__ sz, int nq, double *__restrict__ box)
{
    __shared__ double red[6][kRun];
    const int i = blockIdx.x * kRun + threadIdx.x;
    const int i0 = blockIdx.x * kRun;
    const bool act = i < nq;
    const double v[3] = {act ? sx[i] : sx[i0], act ? sy[i] : sy[i0], act ? sz[i] : sz[i0]};
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = v[k];
        red[3 + k][threadIdx.x] = v[k];
    }
    __syncthreads();
    for (int h = kRun / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 6; ++k)
                red[k][threadIdx.x] = k < 3 ? fmin(red[k][threadIdx.x], red[k][threadIdx.x + h])
                                            : fmax(red[k][threadIdx.x], red[k][threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x < 6) box[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// E at every charge from all other charges, over charges in Morton order
// (positions sx/sy/sz, charges sq, all sorted; 64-charge boxes from
// k_tile_boxes); written to the sorted outputs ox/oy/oz, scaled by k_e.
__global__ __launch_bounds__(kCB) void k_coulomb_sorted(const double *__restrict__ sx, const double *__restrict__ sy,
                                                        const double *__restrict__ sz, const double *__restrict__ sq,
                                                        const double *__restrict__ box, int nq,
                                                        double *__restrict__ ox, double *__restrict__ oy,
                                                        double *__restrict__ oz)
{
    __shared__ float4 src[kCB];                   // offset from the run's box centre (um), charge
    __shared__ double nx[kCB], ny[kCB], nz[kCB];  // FP64 positions, for the near runs
    const int nbox = (nq + kRun - 1) / kRun;
    const int b0 = blockIdx.x * kCB;
    const int i = b0 + threadIdx.x;
    const bool act = i < nq;
    // lanes past the last charge stand at the block's first charge
    const double xi = act ? sx[i] : sx[b0], yi = act ? sy[i] : sy[b0], zi = act ? sz[i] : sz[b0];
    // the wave's box (wave-uniform, so the near / far choice is a scalar branch)
    const int tbox =
        __builtin_amdgcn_readfirstlane(min((int)(blockIdx.x * (kCB / kRun)) + (int)(threadIdx.x / kRun), nbox - 1));
    const double *mb = box + 6 * (size_t)tbox;
    const double m0 = mb[0], m1 = mb[1], m2 = mb[2], m3 = mb[3], m4 = mb[4], m5 = mb[5];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int base = 0; base < nq; base += kCB) {
        __syncthreads();
        const int j = base + threadIdx.x;
        if (j < nq) {
            const double *jb = box + 6 * (size_t)(j / kRun);
            const double ocx = 0.5 * (jb[0] + jb[3]), ocy = 0.5 * (jb[1] + jb[4]), ocz = 0.5 * (jb[2] + jb[5]);
            src[threadIdx.x] = make_float4((float)((sx[j] - ocx) * kUm), (float)((sy[j] - ocy) * kUm),
                                           (float)((sz[j] - ocz) * kUm), (float)sq[j]);
            nx[threadIdx.x] = sx[j];
            ny[threadIdx.x] = sy[j];
            nz[threadIdx.x] = sz[j];
        } else {  // padding: a zero charge at the box centre / the block's first charge
            src[threadIdx.x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            nx[threadIdx.x] = sx[b0];
            ny[threadIdx.x] = sy[b0];
            nz[threadIdx.x] = sz[b0];
        }
        __syncthreads();
#pragma unroll 1
        for (int r0 = 0; r0 < kCB; r0 += kRun) {
            const int sb = (base + r0) / kRun;  // uniform
            if (sb >= nbox) break;
            const double *tb = box + 6 * (size_t)sb;
            const double gx = fmax(0.0, fmax(tb[0] - m3, m0 - tb[3]));
            const double gy = fmax(0.0, fmax(tb[1] - m4, m1 - tb[4]));
            const double gz = fmax(0.0, fmax(tb[2] - m5, m2 - tb[5]));
            const double g2 = gx * gx + gy * gy + gz * gz;
            const double sd2 = (tb[3] - tb[0]) * (tb[3] - tb[0]) + (tb[4] - tb[1]) * (tb[4] - tb[1]) +
                               (tb[5] - tb[2]) * (tb[5] - tb[2]);
            if (g2 == 0.0 || g2 < sd2) {  // near (uniform per wave)
                float fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll 8
                for (int k = r0; k < r0 + kRun; ++k) {
                    const float dx = (float)((xi - nx[k]) * kUm);
                    const float dy = (float)((yi - ny[k]) * kUm);
                    const float dz = (float)((zi - nz[k]) * kUm);
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    // the target itself and coincident charges add nothing
                    const float ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                    const float w = (src[k].w * ir) * (ir * ir);
                    fx = fmaf(w, dx, fx);
                    fy = fmaf(w, dy, fy);
                    fz = fmaf(w, dz, fz);
                }
                ax += (double)fx;
                ay += (double)fy;
                az += (double)fz;
                continue;
            }
            // far: the target's offset from this run's box centre
            const float tx = (float)((xi - 0.5 * (tb[0] + tb[3])) * kUm);
            const float ty = (float)((yi - 0.5 * (tb[1] + tb[4])) * kUm);
            const float tz = (float)((zi - 0.5 * (tb[2] + tb[5])) * kUm);
            float fx[8], fy[8], fz[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) fx[u] = fy[u] = fz[u] = 0.0f;
#pragma unroll 1
            for (int g = r0; g < r0 + kRun; g += 8) {
                float4 cs[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) cs[u] = src[g + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float4 c = cs[u];
                    const float dx = tx - c.x, dy = ty - c.y, dz = tz - c.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, kSeedR2)));
                    const float ir = __builtin_amdgcn_rsqf(r2);
                    const float w = (c.w * ir) * (ir * ir);
                    fx[u] = fmaf(w, dx, fx[u]);
                    fy[u] = fmaf(w, dy, fy[u]);
                    fz[u] = fmaf(w, dz, fz[u]);
                }
            }
            ax += (double)(((fx[0] + fx[1]) + (fx[2] + fx[3])) + ((fx[4] + fx[5]) + (fx[6] + fx[7])));
            ay += (double)(((fy[0] + fy[1]) + (fy[2] + fy[3])) + ((fy[4] + fy[5]) + (fy[6] + fy[7])));
            az += (double)(((fz[0] + fz[1]) + (fz[2] + fz[3])) + ((fz[4] + fz[5]) + (fz[6] + fz[7])));
        }
    }
    if (act) {
        // um offsets: q dx / r^3 in C / um^2 -> x 1e12 for C / m^2
        const double sc = kKe * kUm * kUm;
        ox[i] = sc * ax;
        oy[i] = sc * ay;
        oz[i] = sc * az;
    }
}

// e_c[perm[k]] += src[c nq + k]
__global__ __launch_bounds__(kCB) void k_scatter_add3(const double *__restrict__ src, const int *__restrict__ perm,
                                                      int nq, double *__restrict__ ex, double *__restrict__ ey,
                                                      double *__restrict__ ez)
{
    const int k = blockIdx.x * kCB + threadIdx.x;
    if (k >= nq) return;
    const int i = perm[k];
    const size_t n = (size_t)nq;
    ex[i] += src[k];
    ey[i] += src[n + k];
    ez[i] += src[2 * n + k];
}

__global__ __launch_bounds__(kCB) void k_gather1(const double *__restrict__ v, const int *__restrict__ perm, int nq,
                                                 double *__restrict__ out)
{
    const int k = blockIdx.x * kCB + threadIdx.x;
    if (k < nq) out[k] = v[perm[k]];
}

// phi and E of point charges (sources) at arbitrary points (targets),
// added to phi/ex/ey/ez (any may be null): one lane per target, sources
// through LDS; the difference in FP64, the pair term in FP32, runs of 64
// sources summed in FP32 then added to FP64.  Coincident points add nothing.
__global__ __launch_bounds__(kCB) void k_point_field(const double *__restrict__ tx, const double *__restrict__ ty,
                                                     const double *__restrict__ tz, int m,
                                                     const double *__restrict__ qx, const double *__restrict__ qy,
                                                     const double *__restrict__ qz, const double *__restrict__ q,
                                                     int nq, double *__restrict__ phi, double *__restrict__ ex,
                                                     double *__restrict__ ey, double *__restrict__ ez)
{
    __shared__ double sx[kCB], sy[kCB], sz[kCB];
    __shared__ float sq[kCB];
    const int i = blockIdx.x * kCB + threadIdx.x;
    const bool act = i < m;
    const double xi = act ? tx[i] : 0.0, yi = act ? ty[i] : 0.0, zi = act ? tz[i] : 0.0;
    double ap = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int base = 0; base < nq; base += kCB) {
        __syncthreads();
        const int j = base + threadIdx.x;
        sx[threadIdx.x] = j < nq ? qx[j] : 0.0;
        sy[threadIdx.x] = j < nq ? qy[j] : 0.0;
        sz[threadIdx.x] = j < nq ? qz[j] : 0.0;
        sq[threadIdx.x] = j < nq ? (float)q[j] : 0.0f;
        __syncthreads();
#pragma unroll 1
        for (int r0 = 0; r0 < kCB; r0 += kRun) {
            float fp = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll 8
            for (int k = r0; k < r0 + kRun; ++k) {
                const float dx = (float)(xi - sx[k]);
                const float dy = (float)(yi - sy[k]);
                const float dz = (float)(zi - sz[k]);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                const float w = sq[k] * ir;
                fp += w;
                const float w3 = w * (ir * ir);
                fx = fmaf(w3, dx, fx);
                fy = fmaf(w3, dy, fy);
                fz = fmaf(w3, dz, fz);
            }
            ap += (double)fp;
            ax += (double)fx;
            ay += (double)fy;
            az += (double)fz;
        }
    }
    if (act) {
        if (phi) phi[i] += kKe * ap;
        if (ex) ex[i] += kKe * ax;
        if (ey) ey[i] += kKe * ay;
        if (ez) ez[i] += kKe * az;
    }
}

// part[b] = sum of |q| over a strided share of the charges (b < gridDim.x),
// reduced in a fixed order within the block
__global__ __launch_bounds__(kCB) void k_abs_sum(const double *__restrict__ q, int nq, double *__restrict__ part)
{
    __shared__ double red[kCB];
    double a = 0.0;
    for (int i = blockIdx.x * kCB + threadIdx.x; i < nq; i += gridDim.x * kCB) a += fabs(q[i]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int h = kCB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
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


static size_t align256c(size_t b) { return (b + 255) & ~(size_t)255; }

size_t coulomb_workspace(int64_t nq)
{
    if (nq <= 0) return 0;
    const size_t w = order_points_workspace(nq);
    if (!w) return 0;
    const size_t n = (size_t)nq;
    return w + align256c(4 * n) + align256c(24 * n) + align256c(8 * n) + align256c(24 * n) +
           align256c(48 * (size_t)runs(nq));
}

hipError_t launch_coulomb(const double *qx, const double *qy, const double *qz, const double *q, int64_t nq,
                          double *ex, double *ey, double *ez, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    const size_t w0 = order_points_workspace(nq);
    if (!w0 || !ws || ws_bytes < coulomb_workspace(nq)) return hipErrorInvalidValue;
    const size_t n = (size_t)nq;
    char *w = static_cast<char *>(ws);
    int *perm = reinterpret_cast<int *>(w + w0);
    double *sp = reinterpret_cast<double *>(w + w0 + align256c(4 * n));
    double *sq = reinterpret_cast<double *>(w + w0 + align256c(4 * n) + align256c(24 * n));
    double *se = reinterpret_cast<double *>(w + w0 + align256c(4 * n) + align256c(24 * n) + align256c(8 * n));
    double *bx = reinterpret_cast<double *>(w + w0 + align256c(4 * n) + align256c(24 * n) + align256c(8 * n) +
                                            align256c(24 * n));
    hipError_t e = launch_order_points(qx, qy, qz, nq, sp, sp + n, sp + 2 * n, perm, ws, w0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather1, dim3(blocks(nq)), dim3(kCB), 0, s, q, perm, (int)nq, sq);
    hipLaunchKernelGGL(k_tile_boxes, dim3(runs(nq)), dim3(kRun), 0, s, sp, sp + n, sp + 2 * n, (int)nq, bx);
    hipLaunchKernelGGL(k_coulomb_sorted, dim3(blocks(nq)), dim3(kCB), 0, s, sp, sp + n, sp + 2 * n, sq, bx, (int)nq,
                       se, se + n, se + 2 * n);
    hipLaunchKernelGGL(k_scatter_add3, dim3(blocks(nq)), dim3(kCB), 0, s, se, perm, (int)nq, ex, ey, ez);
    return hipGetLastError();
}

void launch_point_field(const double *tx, const double *ty, const double *tz, int64_t m, const double *qx,
                        const double *qy, const double *qz, const double *q, int64_t nq, double *phi, double *ex,
                        double *ey, double *ez, hipStream_t s)
{
    if (m <= 0 || nq <= 0) return;
    hipLaunchKernelGGL(k_point_field, dim3(blocks(m)), dim3(kCB), 0, s, tx, ty, tz, (int)m, qx, qy, qz, q, (int)nq,
                       phi, ex, ey, ez);
}

int launch_abs_sum(const double *q, int64_t nq, double *part, hipStream_t s)
{
    if (nq <= 0) return 0;
    const int nb = (int)std::min<int64_t>(kAbsParts, (nq + kCB - 1) / kCB);
    hipLaunchKernelGGL(k_abs_sum, dim3(nb), dim3(kCB), 0, s, q, (int)nq, part);
    return nb;
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
