// lu_kernels.hip -- dense LU factorisation with row pivoting and triangular
// solves on gfx950 (paper Eq. Matrix, K sigma = phi, and Algorithm 1's LU
// factorisation; the inverse is never formed, new right-hand sides use the
// resident factors).
//
// Blocked right-looking factorisation, column-major A with leading
// dimension n, in two levels: outer blocks of kOuterNB columns, each
// factored by panels of kNB columns whose updates stay inside the outer
// block, followed by one update of the rest of the matrix with the whole
// outer block (K = kOuterNB), so the trailing matrix is read and written
// once per outer block instead of once per panel:
//   for each outer block [K0, K1):
//     for each panel [k, k+kb) of it:
//       1. panel factorisation, one launch per column: every workgroup owns
//          256 consecutive rows; a launch eliminates column c on its rows
//          (scale by the pivot, rank-1 update of the rest of the panel) and
//          then finds the largest |a| of column c+1 among its rows; the last
//          workgroup to finish (atomic counter, no spinning) reduces the
//          per-workgroup maxima, records the pivot (first index among equal
//          maxima) and swaps the two rows inside the panel;
//       2. the same row swaps applied to every column outside the panel;
//       3. U = L11^-1 A for the columns [k+kb, K1) (unit lower solve, LDS);
//       4. A -= L21 U on rows [k+kb, n) x columns [k+kb, K1) (MFMA);
//     5. U12 = L11^-1 A12 for the columns [K1, n), panel by panel (step 3 and
//        an MFMA update of the outer block's lower rows);
//     6. A22 -= L21 U12 on rows and columns [K1, n), K = K1 - K0 (MFMA).
// T = double uses v_mfma_f64_16x16x4_f64, T = float v_mfma_f32_16x16x4_f32.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "lu_internal.hpp"

namespace nebem {

constexpr int kPB = 256;  // rows per panel workgroup

// ------------------------------------------------------------- panel step
// c: column eliminated by this launch (c == k - 1: none, pivot search only).
template <typename T>
__global__ __launch_bounds__(kPB) void k_panel(T *__restrict__ A, int n, int k, int kb, int c,
                                               int *__restrict__ ipiv, T *__restrict__ pval,
                                               int *__restrict__ pidx, int *__restrict__ counter,
                                               int *__restrict__ info)
{
    __shared__ T urow[kNB];
    __shared__ T red_v[kPB];
    __shared__ int red_i[kPB];
    __shared__ int am_last;
    const int tid = threadIdx.x;
    const int r = k + blockIdx.x * kPB + tid;
    const int kend = k + kb;
    const int cn = c + 1;  // column whose pivot is searched
    T vnext = T(0);
    if (c >= k) {
        if (tid < kend - c) urow[tid] = A[(size_t)(c + tid) * n + c];
        __syncthreads();
        const T piv = urow[0];
        if (r > c && r < n) {
            T l = A[(size_t)c * n + r];
            l = (piv != T(0)) ? l / piv : l;
            A[(size_t)c * n + r] = l;
            for (int cc = c + 1; cc < kend; ++cc) {
                T v = A[(size_t)cc * n + r];
                v = v - l * urow[cc - c];
                A[(size_t)cc * n + r] = v;
                if (cc == cn) vnext = v;
            }
        }
    } else if (r < n && cn < kend) {
        vnext = A[(size_t)cn * n + r];
    }
    if (cn >= kend) return;  // last column of the panel: nothing to search
    // block argmax of |A[r, cn]| over r >= cn (first index among equal maxima)
    const bool valid = r >= cn && r < n;
    red_v[tid] = valid ? fabs(vnext) : T(-1);
    red_i[tid] = valid ? r : 0x7fffffff;
    __syncthreads();
    for (int s = kPB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const T a = red_v[tid], b = red_v[tid + s];
            const int ia = red_i[tid], ib = red_i[tid + s];
            if (b > a || (b == a && ib < ia)) {
                red_v[tid] = b;
                red_i[tid] = ib;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        pval[blockIdx.x] = red_v[0];
        pidx[blockIdx.x] = red_i[0];
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) am_last = (atomicAdd(counter, 1) == (int)gridDim.x - 1);
    __syncthreads();
    if (!am_last) return;
    __threadfence();
    // last workgroup: reduce the per-workgroup maxima
    T bv = T(-1);
    int bi = 0x7fffffff;
    for (int b = tid; b < (int)gridDim.x; b += kPB) {
        const T v = pval[b];
        const int i = pidx[b];
        if (v > bv || (v == bv && i < bi)) {
            bv = v;
            bi = i;
        }
    }
    red_v[tid] = bv;
    red_i[tid] = bi;
    __syncthreads();
    for (int s = kPB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const T a = red_v[tid], b = red_v[tid + s];
            const int ia = red_i[tid], ib = red_i[tid + s];
            if (b > a || (b == a && ib < ia)) {
                red_v[tid] = b;
                red_i[tid] = ib;
            }
        }
        __syncthreads();
    }
    int p = red_i[0];
    const T pv = red_v[0];
    if (p < cn || p >= n) p = cn;  // no usable pivot (column all NaN): no swap, flagged below
    if (tid == 0) {
        ipiv[cn] = p;
        if (!(pv > T(0))) atomicMin(info, cn);
        *counter = 0;
    }
    if (p != cn && tid < kb) {
        const size_t col = (size_t)(k + tid) * n;
        const T a = A[col + cn], b = A[col + p];
        A[col + cn] = b;
        A[col + p] = a;
    }
}

// Row swaps of panel [k, k+kb) applied to every column outside the panel.
template <typename T>
__global__ __launch_bounds__(256) void k_laswp(T *__restrict__ A, int n, int k, int kb,
                                               const int *__restrict__ ipiv)
{
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n - kb) return;
    if (j >= k) j += kb;
    T *col = A + (size_t)j * n;
    for (int t = 0; t < kb; ++t) {
        const int p = ipiv[k + t];
        if (p != k + t) {
            const T a = col[k + t];
            col[k + t] = col[p];
            col[p] = a;
        }
    }
}

// U = L11^-1 A[k:k+kb, j] for the columns j in [jb, je), 64 per workgroup
// (unit lower L11 = A[k:k+kb, k:k+kb], kb <= 64).
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(T *__restrict__ A, int n, int k, int kb, int jb, int je)
{
    __shared__ T L[kNB][kNB + 1];
    __shared__ T X[kNB][kNB + 1];
    const int tid = threadIdx.x;
    const int j0 = jb + blockIdx.x * 64;
    const int ncol = min(64, je - j0);
    for (int e = tid; e < kb * kb; e += 256) {
        const int rr = e % kb, cc = e / kb;
        L[rr][cc] = A[(size_t)(k + cc) * n + k + rr];
    }
    for (int e = tid; e < kb * ncol; e += 256) {
        const int rr = e % kb, cc = e / kb;
        X[rr][cc] = A[(size_t)(j0 + cc) * n + k + rr];
    }
    __syncthreads();
    for (int i = 0; i < kb - 1; ++i) {
        for (int e = tid; e < (kb - 1 - i) * ncol; e += 256) {
            const int rr = i + 1 + e % (kb - 1 - i), cc = e / (kb - 1 - i);
            X[rr][cc] -= L[rr][i] * X[i][cc];
        }
        __syncthreads();
    }
    for (int e = tid; e < kb * ncol; e += 256) {
        const int rr = e % kb, cc = e / kb;
        A[(size_t)(j0 + cc) * n + k + rr] = X[rr][cc];
    }
}

// ------------------------------------------------------------------ GEMM
// C -= L21 U12 over the trailing matrix rows/cols [k+kb, n), K = kb <= 64.
// Workgroup tile 64 x 64, four waves each 32 x 32 (2 x 2 MFMA tiles).  The
// MFMA computes the transposed tile, D'[i][j] = C[row j][col i], so that the
// 16 lanes holding one output column walk 16 consecutive rows (contiguous in
// the column-major matrix).  MFMA 16x16x4 operand layout (wave64, checked
// on gfx950): A operand (16 x 4) element [i][kk] in lane i + 16 kk; B operand
// (4 x 16) element [kk][j] in lane j + 16 kk; result element [i][j] in lane
// j + 16 (i / 4), register i % 4 for f32, but lane j + 16 (i % 4), register
// i / 4 for f64.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// result row i held by (lane group g = lane / 16, register v)
template <typename T>
struct Acc;
template <>
struct Acc<double> {
    typedef d4 type;
    static __device__ __forceinline__ int row(int g, int v) { return 4 * v + g; }
};
template <>
struct Acc<float> {
    typedef f4 type;
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};

constexpr int kGT = 64;     // trailing-update workgroup tile (rows and columns)
constexpr int kKC = 32;     // K chunk staged in LDS at a time (keeps several workgroups per CU)
constexpr int kXCD = 8;     // accelerator complex dies; workgroups are dealt to them round-robin
constexpr int kGroupR = 8;  // tile rows per group of the tile order

// C[r0:r1, c0:c1] -= A[r0:r1, k:k+kb] A[k:k+kb, c0:c1] for any kb.  1-D grid
// of kXCD * per_xcd workgroups: workgroup b works on linear tile
// (b % kXCD) * per_xcd + b / kXCD, so each die takes one contiguous range of
// the tile order, and that order walks groups of kGroupR tile rows column by
// column -- the workgroups a die runs at one time share their L21 and U12
// tiles in its L2.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_update(T *__restrict__ A, int n, int k, int kb, int r0, int r1, int c0,
                                                     int c1, int per_xcd)
{
    typedef typename Acc<T>::type V4;
    // One K chunk of the operands.  Strides chosen so that the 32 lanes of
    // each half-wave hit distinct LDS banks on the staging stores and on the
    // MFMA operand loads: -L21 row-major in k (rows contiguous, as in A),
    // U12 column-major (k contiguous, as in A).
    __shared__ T sL[kKC][kGT + 16];  // sL[kk][row] = -L21
    __shared__ T sU[kGT][kKC + 2];   // sU[col][kk] =  U12
    const int nt_r = (r1 - r0 + kGT - 1) / kGT, nt_c = (c1 - c0 + kGT - 1) / kGT;
    const int lin = (int)(blockIdx.x % kXCD) * per_xcd + (int)(blockIdx.x / kXCD);
    if (lin >= nt_r * nt_c) return;  // whole workgroup: padding of the last die's range
    const int gsz = kGroupR * nt_c;
    const int first = (lin / gsz) * kGroupR;
    const int rows_in = min(kGroupR, nt_r - first);
    const int within = lin % gsz;
    const int row0 = r0 + (first + within % rows_in) * kGT;
    const int col0 = c0 + (within / rows_in) * kGT;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;  // wave's 32x32 sub-tile
    const int li = lane & 15, lk = lane >> 4;
    // The accumulators start from C itself (loads issued before the operand
    // staging so that the two overlap); the MFMA chain then adds (-L21) U12.
    V4 acc[2][2];
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gc = col0 + wc + 16 * tc + Acc<T>::row(lk, v);
                const int gr = row0 + wr + 16 * tr + li;
                acc[tc][tr][v] = (gc < c1 && gr < r1) ? A[(size_t)gc * n + gr] : T(0);
            }
    // K in chunks of kKC; entries past kb are staged as zeros, so every chunk
    // has the same compile-time shape (index arithmetic by shifts, the MFMA
    // loop fully unrolled)
    for (int k0 = 0; k0 < kb; k0 += kKC) {
        if (k0) __syncthreads();
#pragma unroll
        for (int e = tid; e < kKC * kGT; e += 256) {
            const int rr = e % kGT, kk = e / kGT;
            const int gr = row0 + rr, gk = k0 + kk;
            sL[kk][rr] = (gr < r1 && gk < kb) ? -A[(size_t)(k + gk) * n + gr] : T(0);
        }
#pragma unroll
        for (int e = tid; e < kKC * kGT; e += 256) {
            const int kk = e % kKC, cc = e / kKC;
            const int gc = col0 + cc, gk = k0 + kk;
            sU[cc][kk] = (gc < c1 && gk < kb) ? A[(size_t)gc * n + k + gk] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            // A operand: U12 columns (i index), B operand: -L21 rows (j index)
            const T u0 = sU[wc + li][kk + lk], u1 = sU[wc + 16 + li][kk + lk];
            const T l0 = sL[kk + lk][wr + li], l1 = sL[kk + lk][wr + 16 + li];
            acc[0][0] = mfma16(u0, l0, acc[0][0]);
            acc[0][1] = mfma16(u0, l1, acc[0][1]);
            acc[1][0] = mfma16(u1, l0, acc[1][0]);
            acc[1][1] = mfma16(u1, l1, acc[1][1]);
        }
    }
    // lane holds D'[i][j] for i = Acc::row(lk, v) (column offset), j = li (row offset)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gc = col0 + wc + 16 * tc + Acc<T>::row(lk, v);
                const int gr = row0 + wr + 16 * tr + li;
                if (gc < c1 && gr < r1) A[(size_t)gc * n + gr] = acc[tc][tr][v];
            }
}

template <typename T>
static void gemm_update(T *A, int n, int k, int kb, int r0, int r1, int c0, int c1, hipStream_t s)
{
    if (r1 <= r0 || c1 <= c0 || kb <= 0) return;
    const int tiles = ((r1 - r0 + kGT - 1) / kGT) * ((c1 - c0 + kGT - 1) / kGT);
    const int per_xcd = (tiles + kXCD - 1) / kXCD;
    hipLaunchKernelGGL(k_gemm_update<T>, dim3((unsigned)(per_xcd * kXCD)), dim3(256), 0, s, A, n, k, kb, r0, r1, c0,
                       c1, per_xcd);
}

template <typename T>
static void trsm(T *A, int n, int k, int kb, int jb, int je, hipStream_t s)
{
    if (je <= jb) return;
    hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)((je - jb + 63) / 64)), dim3(256), 0, s, A, n, k, kb, jb, je);
}

// ------------------------------------------------------ triangular solves
// One launch per 64-row block b of a forward (unit lower) or backward (upper)
// substitution (n x nrhs, column-major, ld = n).  X holds the right-hand side
// being reduced; every workgroup re-solves the 64 x 64 diagonal block from X
// (identical arithmetic everywhere), workgroup 0 stores the solved rows into
// Y, and every workgroup subtracts the block's contribution from its own 256
// rows of X on the unsolved side.  Solved rows are never written to X, so no
// workgroup can read a half-updated diagonal block.
template <typename T, typename TX>
__global__ __launch_bounds__(256) void k_trsv_step(const T *__restrict__ LU, int n, TX *__restrict__ X,
                                                   TX *__restrict__ Y, int nrhs, int b0, int bsz, int lower)
{
    __shared__ TX D[64][65];
    __shared__ TX y[64][8];
    const int tid = threadIdx.x;
    for (int rc = 0; rc < nrhs; rc += 8) {
        const int nr = min(8, nrhs - rc);
        __syncthreads();
        for (int e = tid; e < bsz * bsz; e += 256) {
            const int rr = e % bsz, cc = e / bsz;
            D[rr][cc] = (TX)LU[(size_t)(b0 + cc) * n + b0 + rr];
        }
        for (int e = tid; e < bsz * nr; e += 256) {
            const int rr = e % bsz, q = e / bsz;
            y[rr][q] = X[(size_t)(rc + q) * n + b0 + rr];
        }
        __syncthreads();
        // diagonal block: column-oriented substitution, the updates of the
        // remaining rows of step i spread over the threads (row x rhs pairs)
        if (lower) {
            for (int i = 0; i < bsz - 1; ++i) {
                for (int e = tid; e < (bsz - 1 - i) * nr; e += 256) {
                    const int r = i + 1 + e % (bsz - 1 - i), q = e / (bsz - 1 - i);
                    y[r][q] -= D[r][i] * y[i][q];
                }
                __syncthreads();
            }
        } else {
            for (int i = bsz - 1; i >= 0; --i) {
                if (tid < nr) y[i][tid] /= D[i][i];
                __syncthreads();
                for (int e = tid; e < i * nr; e += 256) {
                    const int r = e % i, q = e / i;
                    y[r][q] -= D[r][i] * y[i][q];
                }
                __syncthreads();
            }
        }
        if (blockIdx.x == 0)
            for (int e = tid; e < bsz * nr; e += 256) {
                const int rr = e % bsz, q = e / bsz;
                Y[(size_t)(rc + q) * n + b0 + rr] = y[rr][q];
            }
        // update rows outside the block on the unsolved side
        const int lo = lower ? b0 + bsz : 0;
        const int hi = lower ? n : b0;
        const int r = lo + blockIdx.x * 256 + tid;
        if (r < hi) {
            for (int q = 0; q < nr; ++q) {
                TX s = X[(size_t)(rc + q) * n + r];
                for (int j = 0; j < bsz; ++j) s -= (TX)LU[(size_t)(b0 + j) * n + r] * y[j][q];
                X[(size_t)(rc + q) * n + r] = s;
            }
        }
    }
}

// X[i] = B[perm[i]] (row gather for the pivoting permutation), nrhs columns
template <typename TB, typename TX>
__global__ __launch_bounds__(256) void k_permute(const TB *__restrict__ B, TX *__restrict__ X,
                                                 const int *__restrict__ perm, int n, int nrhs)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < nrhs; ++q) X[(size_t)q * n + i] = (TX)B[(size_t)q * n + perm[i]];
}

// --------------------------------------------------------------- launchers
template <typename T>
void lu_factor_launch(T *A, int n, int *ipiv, LUWork &w, hipStream_t s)
{
    for (int K0 = 0; K0 < n; K0 += kOuterNB) {
        const int K1 = (n - K0 < kOuterNB) ? n : K0 + kOuterNB;
        for (int k = K0; k < K1; k += kNB) {
            const int kb = (K1 - k < kNB) ? K1 - k : kNB;
            const unsigned gp = (unsigned)((n - k + kPB - 1) / kPB);
            for (int c = k - 1; c < k + kb; ++c)
                hipLaunchKernelGGL(k_panel<T>, dim3(gp), dim3(kPB), 0, s, A, n, k, kb, c, ipiv, (T *)w.pval, w.pidx,
                                   w.counter, w.info);
            if (n - kb > 0) {
                const unsigned gl = (unsigned)((n - kb + 255) / 256);
                hipLaunchKernelGGL(k_laswp<T>, dim3(gl), dim3(256), 0, s, A, n, k, kb, ipiv);
            }
            trsm(A, n, k, kb, k + kb, K1, s);
            gemm_update(A, n, k, kb, k + kb, n, k + kb, K1, s);
        }
        if (K1 < n) {
            for (int b = K0; b < K1; b += kNB) {
                const int bb = (K1 - b < kNB) ? K1 - b : kNB;
                trsm(A, n, b, bb, K1, n, s);
                gemm_update(A, n, b, bb, b + bb, K1, K1, n, s);
            }
            gemm_update(A, n, K0, K1 - K0, K1, n, K1, n, s);
        }
    }
}

// X = A^-1 P B.  W: n x nrhs workspace of type TX.
template <typename T, typename TX>
void lu_solve_launch(const T *LU, int n, const int *perm, const double *B, TX *X, TX *W, int nrhs, hipStream_t s)
{
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((k_permute<double, TX>), dim3(g), dim3(256), 0, s, B, X, perm, n, nrhs);
    for (int b0 = 0; b0 < n; b0 += 64) {  // L W = P B  (X reduced in place, solution in W)
        const int bsz = (n - b0 < 64) ? n - b0 : 64;
        const int rows = n - b0 - bsz;
        const unsigned gb = rows > 0 ? (unsigned)((rows + 255) / 256) : 1u;
        hipLaunchKernelGGL((k_trsv_step<T, TX>), dim3(gb), dim3(256), 0, s, LU, n, X, W, nrhs, b0, bsz, 1);
    }
    const int last = ((n - 1) / 64) * 64;
    for (int b0 = last; b0 >= 0; b0 -= 64) {  // U X = W  (W reduced in place, solution in X)
        const int bsz = (n - b0 < 64) ? n - b0 : 64;
        const int rows = b0;
        const unsigned gb = rows > 0 ? (unsigned)((rows + 255) / 256) : 1u;
        hipLaunchKernelGGL((k_trsv_step<T, TX>), dim3(gb), dim3(256), 0, s, LU, n, W, X, nrhs, b0, bsz, 0);
    }
}

void lu_factor(double *A, int n, int *ipiv, LUWork &w, hipStream_t s) { lu_factor_launch<double>(A, n, ipiv, w, s); }
void lu_factor(float *A, int n, int *ipiv, LUWork &w, hipStream_t s) { lu_factor_launch<float>(A, n, ipiv, w, s); }
void lu_solve(const double *LU, int n, const int *perm, const double *B, double *X, double *W, int nrhs,
              hipStream_t s)
{
    lu_solve_launch<double, double>(LU, n, perm, B, X, W, nrhs, s);
}
void lu_solve(const float *LU, int n, const int *perm, const double *B, float *X, float *W, int nrhs,
              hipStream_t s)
{
    lu_solve_launch<float, float>(LU, n, perm, B, X, W, nrhs, s);
}

}  // namespace nebem
