// refine_kernels.hip -- row equilibration, FP64 residuals and vector helpers
// for the mixed-precision solve (FP32 LU factors + FP64 iterative
// refinement).  The influence matrix mixes rows of very different scale
// (potential rows ~ k_e * size, interface rows ~ 1/eps0), so rows are scaled
// by 1/max_j |A_ij| before the FP32 copy is made; the solution is unchanged.
//
// All reductions are two-pass with a fixed order (partials per column chunk
// or per workgroup, then a sequential sum), so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>

#include "refine_internal.hpp"

namespace nebem {

constexpr int kRB = 256;

// part[c * n + i] = max_{j in chunk c} |A_ij|
__global__ __launch_bounds__(kRB) void k_rowmax_part(const double *__restrict__ A, int n, int chunk,
                                                     double *__restrict__ part)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i >= n) return;
    const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
    double mx = 0.0;
    for (int j = j0; j < j1; ++j) mx = fmax(mx, fabs(A[(size_t)j * n + i]));
    part[(size_t)blockIdx.y * n + i] = mx;
}

__global__ __launch_bounds__(kRB) void k_rowscale(const double *__restrict__ part, int n, int nchunk,
                                                  double *__restrict__ s)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i >= n) return;
    double mx = 0.0;
    for (int c = 0; c < nchunk; ++c) mx = fmax(mx, part[(size_t)c * n + i]);
    s[i] = mx > 0.0 ? 1.0 / mx : 1.0;
}

// A32 = float(diag(s) A), 8 columns per workgroup row-block
__global__ __launch_bounds__(kRB) void k_convert_scaled(const double *__restrict__ A, const double *__restrict__ s,
                                                        int n, float *__restrict__ A32)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i >= n) return;
    const double si = s[i];
    const int j0 = blockIdx.y * 8, j1 = min(n, j0 + 8);
    for (int j = j0; j < j1; ++j) A32[(size_t)j * n + i] = (float)(si * A[(size_t)j * n + i]);
}

// part[c * n + i] = sum_{j in chunk c} A_ij x_j (chunk <= kGemvChunk)
__global__ __launch_bounds__(kRB) void k_gemv_part(const double *__restrict__ A, int n,
                                                   const double *__restrict__ x, double *__restrict__ part)
{
    __shared__ double xs[kGemvChunk];
    const int j0 = blockIdx.y * kGemvChunk, j1 = min(n, j0 + kGemvChunk);
    for (int j = j0 + threadIdx.x; j < j1; j += kRB) xs[j - j0] = x[j];
    __syncthreads();
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) acc = fma(A[(size_t)j * n + i], xs[j - j0], acc);
    part[(size_t)blockIdx.y * n + i] = acc;
}

// ru = b - sum_c part_c ; rs = s .* ru ; sq[blockIdx.x] = sum over the block of ru^2
__global__ __launch_bounds__(kRB) void k_residual(const double *__restrict__ part, int nchunk,
                                                  const double *__restrict__ b, const double *__restrict__ s, int n,
                                                  double *__restrict__ rs, double *__restrict__ sq)
{
    __shared__ double red[kRB];
    const int i = blockIdx.x * kRB + threadIdx.x;
    double r = 0.0;
    if (i < n) {
        double ax = 0.0;
        for (int c = 0; c < nchunk; ++c) ax += part[(size_t)c * n + i];
        r = b[i] - ax;
        rs[i] = s[i] * r;
    }
    red[threadIdx.x] = r * r;
    __syncthreads();
    for (int k = kRB / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) sq[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kRB) void k_sumsq(const double *__restrict__ v, int n, double *__restrict__ sq)
{
    __shared__ double red[kRB];
    const int i = blockIdx.x * kRB + threadIdx.x;
    const double x = i < n ? v[i] : 0.0;
    red[threadIdx.x] = x * x;
    __syncthreads();
    for (int k = kRB / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) sq[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kRB) void k_add_f32(double *__restrict__ x, const float *__restrict__ d, int n)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i < n) x[i] += (double)d[i];
}

__global__ __launch_bounds__(kRB) void k_add_f64(double *__restrict__ x, const double *__restrict__ d, int n)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i < n) x[i] += d[i];
}

__global__ __launch_bounds__(kRB) void k_scale_vec(const double *__restrict__ s, const double *__restrict__ b,
                                                   int n, double *__restrict__ out)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i < n) out[i] = s[i] * b[i];
}

__global__ __launch_bounds__(kRB) void k_fill(double *__restrict__ x, int n, double v)
{
    const int i = blockIdx.x * kRB + threadIdx.x;
    if (i < n) x[i] = v;
}

static inline unsigned blocks(int n) { return (unsigned)((n + kRB - 1) / kRB); }

void row_scale(const double *A, int n, double *part, double *s, hipStream_t st)
{
    const int nchunk = (n + kRowChunk - 1) / kRowChunk;
    hipLaunchKernelGGL(k_rowmax_part, dim3(blocks(n), nchunk), dim3(kRB), 0, st, A, n, kRowChunk, part);
    hipLaunchKernelGGL(k_rowscale, dim3(blocks(n)), dim3(kRB), 0, st, part, n, nchunk, s);
}

void convert_scaled(const double *A, const double *s, int n, float *A32, hipStream_t st)
{
    hipLaunchKernelGGL(k_convert_scaled, dim3(blocks(n), (n + 7) / 8), dim3(kRB), 0, st, A, s, n, A32);
}

void residual(const double *A, int n, const double *x, const double *b, const double *s, double *part, double *rs,
              double *sq, hipStream_t st)
{
    const int nchunk = (n + kGemvChunk - 1) / kGemvChunk;
    hipLaunchKernelGGL(k_gemv_part, dim3(blocks(n), nchunk), dim3(kRB), 0, st, A, n, x, part);
    hipLaunchKernelGGL(k_residual, dim3(blocks(n)), dim3(kRB), 0, st, part, nchunk, b, s, n, rs, sq);
}

void sumsq(const double *v, int n, double *sq, hipStream_t st)
{
    hipLaunchKernelGGL(k_sumsq, dim3(blocks(n)), dim3(kRB), 0, st, v, n, sq);
}

void add_f32(double *x, const float *d, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_add_f32, dim3(blocks(n)), dim3(kRB), 0, st, x, d, n);
}

// cs[j] = sum_i |A_ij| (column j of the column-major matrix), one workgroup
// per column, fixed-order reduction
__global__ __launch_bounds__(kRB) void k_colabs(const double *__restrict__ A, int n, double *__restrict__ cs)
{
    __shared__ double red[kRB];
    const int j = blockIdx.x;
    const double *col = A + (size_t)j * n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kRB) acc += fabs(col[i]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int sft = kRB / 2; sft > 0; sft >>= 1) {
        if ((int)threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
        __syncthreads();
    }
    if (threadIdx.x == 0) cs[j] = red[0];
}

void column_abs_sums(const double *A, int n, double *cs, hipStream_t st)
{
    hipLaunchKernelGGL(k_colabs, dim3((unsigned)n), dim3(kRB), 0, st, A, n, cs);
}

void add_f64(double *x, const double *d, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_add_f64, dim3(blocks(n)), dim3(kRB), 0, st, x, d, n);
}

void scale_vec(const double *s, const double *b, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_vec, dim3(blocks(n)), dim3(kRB), 0, st, s, b, n, out);
}

void fill(double *x, int n, double v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks(n)), dim3(kRB), 0, st, x, n, v);
}

}  // namespace nebem
