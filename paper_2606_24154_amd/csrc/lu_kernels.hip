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
//       1. panel factorisation: every workgroup owns 256 consecutive rows.
//          Normally one cooperative launch for the whole panel, the rows kept
//          in LDS and the columns separated by grid barriers (k_panel_fused);
//          if the device cannot hold all of the panel's workgroups at once,
//          one launch per column: a launch eliminates column c on its rows
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
#include <climits>
#include <cstdlib>
#include <cmath>

#include "lu_internal.hpp"

namespace nebem {

constexpr int kPB = 256;  // rows per panel workgroup

// Lane i's value broadcast to the wave (i uniform): v_readlane, no LDS.
__device__ __forceinline__ double lane_bcast(double v, int i)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bcast(float v, int i)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}

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
            // the row's entries in columns c .. kend-1 are loaded 32 at a time
            // and all in flight together
            T l = A[(size_t)c * n + r];
            for (int c0 = c + 1; c0 < kend; c0 += 32) {
                T v[32];
#pragma unroll
                for (int t = 0; t < 32; ++t) v[t] = (c0 + t < kend) ? A[(size_t)(c0 + t) * n + r] : T(0);
                if (c0 == c + 1) {
                    l = (piv != T(0)) ? l / piv : l;
                    A[(size_t)c * n + r] = l;
                }
#pragma unroll
                for (int t = 0; t < 32; ++t)
                    if (c0 + t < kend) {
                        const T w = v[t] - l * urow[c0 + t - c];
                        A[(size_t)(c0 + t) * n + r] = w;
                        if (c0 + t == cn) vnext = w;
                    }
            }
            if (c + 1 >= kend) {
                l = (piv != T(0)) ? l / piv : l;
                A[(size_t)c * n + r] = l;
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

// --------------------------------------------- single-launch panel
// The whole panel [k, k+kb) x rows [k, n) factored by one cooperative launch
// (all G workgroups resident at once): workgroup b keeps its 256 rows of the
// panel in LDS for all kb columns, and the columns are separated by grid
// barriers instead of launches.  Per column c:
//   1. each workgroup finds its candidate (largest |a_rc|, r >= c, first
//      index among equal maxima) and publishes it with the candidate's row;
//      the owner of row c publishes row c;
//   2. grid barrier;
//   3. every workgroup reduces the G candidates in the same total order, so
//      all agree on the pivot row p, takes p's entries as the U row, swaps
//      rows c and p if it owns either, and eliminates column c on its rows.
// Published values are double-buffered by column parity: a slot is written
// again two columns later, after a barrier that every reader of it has
// passed.  Each barrier wait is bounded (kSpinLimit polls, well under a
// second); a wait that gives up sets *timeout, and every later wait of the
// factorisation that sees the flag returns at once, so the launches run to
// their end and the host reports an error instead of the device hanging.
constexpr unsigned kSpinLimit = 1u << 17;

template <typename T>
__device__ __forceinline__ void argmax_take(T &v, int &i, T v2, int i2)
{
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

// (largest value, smallest index among equal) over the workgroup; every
// thread receives the result.  sv, si: kPB/64 entries of LDS.
template <typename T>
__device__ __forceinline__ void block_argmax(T &v, int &i, T *sv, int *si)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const T v2 = __shfl_xor(v, off);
        const int i2 = __shfl_xor(i, off);
        argmax_take(v, i, v2, i2);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = v;
        si[threadIdx.x >> 6] = i;
    }
    __syncthreads();
    v = sv[0];
    i = si[0];
#pragma unroll
    for (int q = 1; q < kPB / 64; ++q) argmax_take(v, i, sv[q], si[q]);
}

// The workgroup barrier completes every wave's stores to L2 (write-through
// L1); thread 0's agent-scope fences then write L2 back for the other dies
// before it arrives, and invalidate the CU's caches after the wait.
__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned target, int *timeout)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(bar, 1u);
        unsigned polls = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            __builtin_amdgcn_s_sleep(2);
            if (++polls == kSpinLimit) {
                atomicExch(timeout, 1);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kPB) void k_panel_fused(T *__restrict__ A, int n, int k, int kb, int *__restrict__ ipiv,
                                                     int *__restrict__ info, T *__restrict__ cval,
                                                     int *__restrict__ cidx, T *__restrict__ crow,
                                                     T *__restrict__ trow, unsigned *__restrict__ bar,
                                                     int *__restrict__ timeout, unsigned base)
{
    __shared__ T S[kNB * kPB];  // this workgroup's rows of the panel, S[col * kPB + row]
    __shared__ T urow[kNB];
    __shared__ T sv[kPB / 64];
    __shared__ int si[kPB / 64];
    const int t = threadIdx.x, b = blockIdx.x, G = gridDim.x;
    const int r = k + b * kPB + t;
    const bool live = r < n;
    for (int j0 = 0; j0 < kb; j0 += 16) {  // 16 loads in flight per thread
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = (live && j0 + u < kb) ? A[(size_t)(k + j0 + u) * n + r] : T(0);
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (j0 + u < kb) S[(j0 + u) * kPB + t] = v[u];
    }
    for (int j = 0; j < kb; ++j) {
        const int c = k + j, sl = j & 1;
        // 1. this workgroup's candidate (a NaN entry never wins)
        const T x = fabs(S[j * kPB + t]);
        const bool valid = live && r >= c;
        T v = (valid && x == x) ? x : T(-1);
        int i = valid ? r : INT_MAX;
        block_argmax(v, i, sv, si);
        if (t == 0) {
            cval[sl * G + b] = v;
            cidx[sl * G + b] = i;
        }
        // the candidate's row and row c, one entry per thread
        const int il = i - k - b * kPB;  // candidate's slot in S (i valid: 0 <= il < kPB)
        if (i != INT_MAX && t < kb) crow[((size_t)sl * G + b) * kNB + t] = S[t * kPB + il];
        const int cl = c - k - b * kPB;
        if (cl >= 0 && cl < kPB && t < kb) trow[sl * kNB + t] = S[t * kPB + cl];
        // 2. every candidate published
        grid_barrier(bar, base + (unsigned)(j + 1) * (unsigned)G, timeout);
        // 3. pivot, row swap, elimination
        T pv = T(-1);
        int p = INT_MAX;
        for (int g = t; g < G; g += kPB) argmax_take(pv, p, cval[sl * G + g], cidx[sl * G + g]);
        block_argmax(pv, p, sv, si);
        if (p < c || p >= n) p = c;
        const int bw = (p - k) / kPB;
        if (t < kb) urow[t] = (p == c) ? trow[sl * kNB + t] : crow[((size_t)sl * G + bw) * kNB + t];
        __syncthreads();
        if (p != c) {
            if (r == c)
                for (int jj = 0; jj < kb; ++jj) S[jj * kPB + t] = urow[jj];
            else if (r == p)
                for (int jj = 0; jj < kb; ++jj) S[jj * kPB + t] = trow[sl * kNB + jj];
        }
        if (b == 0 && t == 0) {
            ipiv[c] = p;
            if (!(pv > T(0))) atomicMin(info, c);
        }
        const T piv = urow[j];
        if (live && r > c) {
            T l = S[j * kPB + t];
            l = (piv != T(0)) ? l / piv : l;
            S[j * kPB + t] = l;
            for (int jj = j + 1; jj < kb; ++jj) S[jj * kPB + t] -= l * urow[jj];
        }
    }
    if (live)
        for (int jj = 0; jj < kb; ++jj) A[(size_t)(k + jj) * n + r] = S[jj * kPB + t];
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
// (unit lower L11 = A[k:k+kb, k:k+kb], kb <= 64).  Wave w solves columns
// 16w .. 16w+15 with lane r holding row r of each: the entry solved at step
// i reaches the other lanes by readlane, so the waves run without barriers;
// every subtraction comes in the order of plain forward substitution.
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(T *__restrict__ A, int n, int k, int kb, int jb, int je)
{
    __shared__ T L[kNB][kNB + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int j0 = jb + blockIdx.x * 64;
    const int ncol = min(64, je - j0);
    T x[16];
    {
        // 16 + 16 loads per thread, all issued before the first is used
        T lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, rr = e & 63, cc = e >> 6;
            lv[u] = (rr < kb && cc < kb) ? A[(size_t)(k + cc) * n + k + rr] : T(0);
            const int xc = 16 * w + u;
            x[u] = (lane < kb && xc < ncol) ? A[(size_t)(j0 + xc) * n + k + lane] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            L[e & 63][e >> 6] = lv[u];
        }
    }
    __syncthreads();
    const bool row_in = lane < kb;
    for (int i = 0; i < kb - 1; ++i) {
        const T l = L[lane][i];
        const bool upd = row_in && lane > i;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const T xi = lane_bcast(x[q], i);
            const T u = x[q] - l * xi;
            x[q] = upd ? u : x[q];
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int xc = 16 * w + q;
        if (row_in && xc < ncol) A[(size_t)(j0 + xc) * n + k + lane] = x[q];
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
    // Every global load is unconditional, from an index clamped into the
    // matrix, and out-of-range entries are replaced when they reach LDS (or
    // are never stored, for C): a load under a branch would have to complete
    // inside that branch, one memory latency per load.
    V4 acc[2][2];
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gc = col0 + wc + 16 * tc + Acc<T>::row(lk, v);
                const int gr = row0 + wr + 16 * tr + li;
                acc[tc][tr][v] = A[(size_t)min(gc, c1 - 1) * n + min(gr, r1 - 1)];
            }
    // K in chunks of kKC; entries past kb are staged as zeros, so every chunk
    // has the same compile-time shape (index arithmetic by shifts, the MFMA
    // loop fully unrolled).  FP32: the next chunk's global loads are issued
    // into registers before the current chunk's MFMAs and stored to LDS
    // after them, so their latency hides behind the matrix-core work.  FP64:
    // the chunk's loads are issued together when it is needed (the prefetch
    // registers would halve the resident workgroups).
    constexpr bool kPrefetch = sizeof(T) == 4;
    constexpr int kPer = kKC * kGT / 256;  // staged entries per thread and operand
    T pl[kPer], pu[kPer];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const int rr = e % kGT, kl = e / kGT;
            pl[u] = A[(size_t)(k + min(k0 + kl, kb - 1)) * n + min(row0 + rr, r1 - 1)];
            const int ku = e % kKC, cc = e / kKC;
            pu[u] = A[(size_t)min(col0 + cc, c1 - 1) * n + k + min(k0 + ku, kb - 1)];
        }
    };
    auto stage = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const int rr = e % kGT, kl = e / kGT;
            sL[kl][rr] = (row0 + rr < r1 && k0 + kl < kb) ? -pl[u] : T(0);
            const int ku = e % kKC, cc = e / kKC;
            sU[cc][ku] = (col0 + cc < c1 && k0 + ku < kb) ? pu[u] : T(0);
        }
    };
    if constexpr (kPrefetch) fetch(0);
    for (int k0 = 0; k0 < kb; k0 += kKC) {
        if (k0) __syncthreads();  // every wave is done reading the previous chunk
        if constexpr (!kPrefetch) fetch(k0);
        stage(k0);
        __syncthreads();
        if constexpr (kPrefetch) {
            if (k0 + kKC < kb) fetch(k0 + kKC);
        }
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

// The same update with 128 x 128 workgroup tiles for large trailing
// matrices: four waves of 64 x 64 (4 x 4 MFMA tiles, 16 accumulators in the
// matrix-core registers), K in chunks of kBK staged through two LDS buffers,
// the next chunk's global loads held in registers while the current chunk's
// MFMAs run, one workgroup barrier per chunk.  Per output element the MFMA
// sequence (accumulator from C, K in steps of 4 in increasing order) is that
// of k_gemm_update, so both give bit-identical results; the larger tile
// halves the operand bytes staged per FLOP.
constexpr int kBT = 128;  // large-update workgroup tile (rows and columns)
constexpr int kBK = 16;   // its K chunk

template <typename T>
__global__ __launch_bounds__(256, 2) void k_gemm_update_big(T *__restrict__ A, int n, int k, int kb, int r0, int r1,
                                                            int c0, int c1, int per_xcd)
{
    typedef typename Acc<T>::type V4;
    // strides as in k_gemm_update: consecutive k of sL, and the 16 columns a
    // half-wave reads from sU, fall on distinct LDS banks
    __shared__ T sL[2][kBK][kBT + 16];  // sL[buf][kk][row] = -L21
    __shared__ T sU[2][kBT][kBK + 2];   // sU[buf][col][kk] =  U12
    const int nt_r = (r1 - r0 + kBT - 1) / kBT, nt_c = (c1 - c0 + kBT - 1) / kBT;
    const int lin = (int)(blockIdx.x % kXCD) * per_xcd + (int)(blockIdx.x / kXCD);
    if (lin >= nt_r * nt_c) return;  // whole workgroup: padding of the last die's range
    const int gsz = kGroupR * nt_c;
    const int first = (lin / gsz) * kGroupR;
    const int rows_in = min(kGroupR, nt_r - first);
    const int within = lin % gsz;
    const int row0 = r0 + (first + within % rows_in) * kBT;
    const int col0 = c0 + (within / rows_in) * kBT;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;  // wave's 64 x 64 sub-tile
    const int li = lane & 15, lk = lane >> 4;
    // Every global load is unconditional, from an index clamped into the
    // matrix, and out-of-range entries are replaced when they reach LDS or
    // the accumulators: a load under a branch would have to complete inside
    // that branch, one memory latency per load.
    V4 acc[4][4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int tr = 0; tr < 4; ++tr)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gc = col0 + wc + 16 * tc + Acc<T>::row(lk, v);
                const int gr = row0 + wr + 16 * tr + li;
                acc[tc][tr][v] = A[(size_t)min(gc, c1 - 1) * n + min(gr, r1 - 1)];
            }
    constexpr int kPer = kBK * kBT / 256;  // staged entries per thread and operand
    T pl[kPer], pu[kPer];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const int rr = e % kBT, kl = e / kBT;
            pl[u] = A[(size_t)(k + min(k0 + kl, kb - 1)) * n + min(row0 + rr, r1 - 1)];
            const int ku = e % kBK, cc = e / kBK;
            pu[u] = A[(size_t)min(col0 + cc, c1 - 1) * n + k + min(k0 + ku, kb - 1)];
        }
    };
    auto stage = [&](int b, int k0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const int rr = e % kBT, kl = e / kBT;
            sL[b][kl][rr] = (row0 + rr < r1 && k0 + kl < kb) ? -pl[u] : T(0);
            const int ku = e % kBK, cc = e / kBK;
            sU[b][cc][ku] = (col0 + cc < c1 && k0 + ku < kb) ? pu[u] : T(0);
        }
    };
    const int nch = (kb + kBK - 1) / kBK;
    fetch(0);
    stage(0, 0);
    if (nch > 1) fetch(kBK);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int b = c & 1;
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 4) {
            T u[4], l[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                u[t] = sU[b][wc + 16 * t + li][kk + lk];
                l[t] = sL[b][kk + lk][wr + 16 * t + li];
            }
#pragma unroll
            for (int tc = 0; tc < 4; ++tc)
#pragma unroll
                for (int tr = 0; tr < 4; ++tr) acc[tc][tr] = mfma16(u[tc], l[tr], acc[tc][tr]);
        }
        // the other buffer was last read in chunk c - 1, which every wave
        // finished before the previous barrier
        if (c + 1 < nch) {
            stage(b ^ 1, (c + 1) * kBK);
            if (c + 2 < nch) fetch((c + 2) * kBK);
        }
        __syncthreads();
    }
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int tr = 0; tr < 4; ++tr)
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
    if (r1 - r0 >= 2 * kBT && c1 - c0 >= 2 * kBT) {
        const int tiles = ((r1 - r0 + kBT - 1) / kBT) * ((c1 - c0 + kBT - 1) / kBT);
        const int per_xcd = (tiles + kXCD - 1) / kXCD;
        hipLaunchKernelGGL(k_gemm_update_big<T>, dim3((unsigned)(per_xcd * kXCD)), dim3(256), 0, s, A, n, k, kb, r0,
                           r1, c0, c1, per_xcd);
        return;
    }
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
// The diagonal block is solved by one wave per right-hand side: lane r holds
// row r, and the entry solved at step i reaches the other lanes by readlane,
// so the 64 sequential steps need no workgroup barrier.  The order of every
// subtraction is that of plain column-oriented substitution.
template <typename T, typename TX>
__global__ __launch_bounds__(256) void k_trsv_step(const T *__restrict__ LU, int n, TX *__restrict__ X,
                                                   TX *__restrict__ Y, int nrhs, int b0, int bsz, int lower)
{
    __shared__ TX D[64][65];
    __shared__ TX y[64][8];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    for (int rc = 0; rc < nrhs; rc += 8) {
        const int nr = min(8, nrhs - rc);
        __syncthreads();
        {
            // all 16 + 2 loads of a thread issued before the first is used
            TX dv[16], yv[2];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = tid + 256 * u, rr = e & 63, cc = e >> 6;
                dv[u] = (rr < bsz && cc < bsz) ? (TX)LU[(size_t)(b0 + cc) * n + b0 + rr] : TX(0);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = tid + 256 * u, rr = e & 63, q = e >> 6;
                yv[u] = (rr < bsz && q < nr) ? X[(size_t)(rc + q) * n + b0 + rr] : TX(0);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = tid + 256 * u;
                D[e & 63][e >> 6] = dv[u];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = tid + 256 * u;
                y[e & 63][e >> 6] = yv[u];
            }
        }
        __syncthreads();
        for (int q = wv; q < nr; q += 4) {
            const bool in = lane < bsz;
            TX v = in ? y[lane][q] : TX(0);
            // the LDS loads do not depend on the substitution: eight of them
            // are issued ahead of each eight steps
            if (lower) {
                for (int i0 = 0; i0 < bsz - 1; i0 += 8) {
                    TX d[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) d[t] = D[lane][i0 + t];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int i = i0 + t;
                        if (i < bsz - 1) {
                            const TX yi = lane_bcast(v, i);
                            const TX u = v - d[t] * yi;
                            v = (in && lane > i) ? u : v;
                        }
                    }
                }
            } else {
                for (int i0 = ((bsz - 1) & ~7); i0 >= 0; i0 -= 8) {
                    TX d[8], dd[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        d[t] = D[lane][i0 + t];
                        dd[t] = D[(i0 + t) & 63][(i0 + t) & 63];
                    }
#pragma unroll
                    for (int t = 7; t >= 0; --t) {
                        const int i = i0 + t;
                        if (i < bsz) {
                            const TX yi = lane_bcast(v, i) / dd[t];
                            const TX u = v - d[t] * yi;
                            v = (lane == i) ? yi : ((in && lane < i) ? u : v);
                        }
                    }
                }
            }
            if (in) y[lane][q] = v;
        }
        __syncthreads();
        if (blockIdx.x == 0)
            for (int e = tid; e < bsz * nr; e += 256) {
                const int rr = e % bsz, q = e / bsz;
                Y[(size_t)(rc + q) * n + b0 + rr] = y[rr][q];
            }
        // update rows outside the block on the unsolved side; each factor
        // entry is loaded once for all right-hand sides of the chunk
        const int lo = lower ? b0 + bsz : 0;
        const int hi = lower ? n : b0;
        const int r = lo + blockIdx.x * 256 + tid;
        if (r < hi) {
            TX acc[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = q < nr ? X[(size_t)(rc + q) * n + r] : TX(0);
            for (int j0 = 0; j0 < bsz; j0 += 16) {
                TX l[16];  // 16 factor entries in flight at once
#pragma unroll
                for (int t = 0; t < 16; ++t) l[t] = (j0 + t < bsz) ? (TX)LU[(size_t)(b0 + j0 + t) * n + r] : TX(0);
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    if (j0 + t < bsz) {
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (q < nr) acc[q] -= l[t] * y[j0 + t][q];
                    }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nr) X[(size_t)(rc + q) * n + r] = acc[q];
        }
    }
}

// Transposed solves with the same factors, one right-hand side, one launch
// per 64-row block: lower = 1 solves U^T w = v forward (U^T lower, diagonal
// of U), lower = 0 solves L^T v = w backward (unit diagonal).  Row r of a
// transposed factor is column r of LU, so the block's entries of row r are
// LU[r n + b0 .. b0 + 63], contiguous.  X is reduced in place on the
// unsolved side and the block's solution goes to Y (as in k_trsv_step).
__global__ __launch_bounds__(256) void k_trsv_t_step(const double *__restrict__ LU, int n, double *__restrict__ X,
                                                     double *__restrict__ Y, int b0, int bsz, int lower)
{
    __shared__ double D[64][65];  // D[r][c] = (transposed factor)[b0 + r][b0 + c]
    __shared__ double y[64];
    const int tid = threadIdx.x;
    {
        double dv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, c = e & 63, r = e >> 6;
            dv[u] = (r < bsz && c < bsz) ? LU[(size_t)(b0 + r) * n + b0 + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            D[e >> 6][e & 63] = dv[u];
        }
        if (tid < 64) y[tid] = tid < bsz ? X[b0 + tid] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {  // one wave: lane r holds row r
        const int lane = tid;
        const bool in = lane < bsz;
        double v = y[lane];
        if (lower) {
            for (int i = 0; i < bsz; ++i) {
                const double yi = lane_bcast(v, i) / D[i][i];
                const double u = v - D[lane][i] * yi;
                v = (lane == i) ? yi : ((in && lane > i) ? u : v);
            }
        } else {
            for (int i = bsz - 1; i >= 0; --i) {
                const double yi = lane_bcast(v, i);
                const double u = v - D[lane][i] * yi;
                v = (in && lane < i) ? u : v;
            }
        }
        if (in) y[lane] = v;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < bsz) Y[b0 + tid] = y[tid];
    const int lo = lower ? b0 + bsz : 0;
    const int hi = lower ? n : b0;
    const int r = lo + blockIdx.x * 256 + tid;
    if (r < hi) {
        double acc = X[r];
        const double *row = LU + (size_t)r * n + b0;
        for (int j0 = 0; j0 < bsz; j0 += 16) {
            double l[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) l[t] = (j0 + t < bsz) ? row[j0 + t] : 0.0;
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (j0 + t < bsz) acc -= l[t] * y[j0 + t];
        }
        X[r] = acc;
    }
}

// z[perm[i]] = v[i] (the inverse of the pivoting gather)
__global__ __launch_bounds__(256) void k_unpermute(const double *__restrict__ v, double *__restrict__ z,
                                                   const int *__restrict__ perm, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) z[perm[i]] = v[i];
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
// Workgroups of k_panel_fused<T> the device holds at once (0 if unknown).
template <typename T>
static int fused_capacity()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_panel_fused<T>, kPB, 0) != hipSuccess) return 0;
    return per_cu * cus;
}

// NEBEM_PANEL_PER_COLUMN=1 in the environment selects the per-column panel
// launches everywhere (the path taken when a panel's workgroups do not fit
// on the device at once), so that tests can reach it at any size.
static bool per_column_forced()
{
    const char *e = std::getenv("NEBEM_PANEL_PER_COLUMN");
    return e && e[0] == '1';
}

template <typename T>
void lu_factor_launch(T *A, int n, int *ipiv, LUWork &w, hipStream_t s)
{
    const int cap = (w.cval && !per_column_forced()) ? fused_capacity<T>() : 0;
    unsigned base = 0;  // barrier arrivals so far (bar starts at 0)
    bool fused_ok = cap > 0;
    for (int K0 = 0; K0 < n; K0 += kOuterNB) {
        const int K1 = (n - K0 < kOuterNB) ? n : K0 + kOuterNB;
        for (int k = K0; k < K1; k += kNB) {
            const int kb = (K1 - k < kNB) ? K1 - k : kNB;
            const unsigned gp = (unsigned)((n - k + kPB - 1) / kPB);
            bool done = false;
            if (fused_ok && (int)gp <= cap) {
                T *cval = (T *)w.cval, *crow = (T *)w.crow, *trow = (T *)w.trow;
                int a_n = n, a_k = k, a_kb = kb;
                void *args[] = {&A,      &a_n,  &a_k,  &a_kb,  &ipiv,      &w.info, &cval,
                                &w.cidx, &crow, &trow, &w.bar, &w.timeout, &base};
                if (hipLaunchCooperativeKernel((const void *)k_panel_fused<T>, dim3(gp), dim3(kPB), args, 0, s) ==
                    hipSuccess) {
                    base += (unsigned)kb * gp;
                    done = true;
                } else {
                    (void)hipGetLastError();
                    fused_ok = false;  // per-column launches from here on
                }
            }
            if (!done)
                for (int c = k - 1; c < k + kb; ++c)
                    hipLaunchKernelGGL(k_panel<T>, dim3(gp), dim3(kPB), 0, s, A, n, k, kb, c, ipiv, (T *)w.pval,
                                       w.pidx, w.counter, w.info);
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

void lu_solve_transposed(const double *LU, int n, const int *perm, const double *b, double *z, double *W,
                         double *V, hipStream_t s)
{
    // U^T w = b: X = W (copy of b, reduced in place), solution in V
    (void)hipMemcpyAsync(W, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
    for (int b0 = 0; b0 < n; b0 += 64) {
        const int bsz = (n - b0 < 64) ? n - b0 : 64;
        const int rows = n - b0 - bsz;
        const unsigned gb = rows > 0 ? (unsigned)((rows + 255) / 256) : 1u;
        hipLaunchKernelGGL(k_trsv_t_step, dim3(gb), dim3(256), 0, s, LU, n, W, V, b0, bsz, 1);
    }
    // L^T v = w: X = V, solution in W
    const int last = ((n - 1) / 64) * 64;
    for (int b0 = last; b0 >= 0; b0 -= 64) {
        const int bsz = (n - b0 < 64) ? n - b0 : 64;
        const unsigned gb = b0 > 0 ? (unsigned)((b0 + 255) / 256) : 1u;
        hipLaunchKernelGGL(k_trsv_t_step, dim3(gb), dim3(256), 0, s, LU, n, V, W, b0, bsz, 0);
    }
    hipLaunchKernelGGL(k_unpermute, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, z, perm, n);
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
