// solver.hip -- host drivers of the dense solve (paper Eq. Matrix and
// Algorithm 1's LU factorisation; Sec. 4.1: factors stay resident and are
// reused for new right-hand sides).
//
// FP64 mode: LU with row pivoting in place, triangular solves.
// Mixed mode: rows equilibrated (s_i = 1/max_j |A_ij|), FP32 copy factored on
// the matrix cores, then classical iterative refinement with FP64 residuals
// (J. H. Wilkinson's scheme; analysed for low-precision factorisations by
// E. Carson and N. J. Higham, SIAM J. Sci. Comput. 40(2):A817-A847, 2018):
//   x_0 = 0;  repeat  d = (S A)_32^-1 S r;  x += d;  r = b - A x  (FP64)
// until ||r||_2 <= tol ||b||_2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "host_util.hpp"
#include "lu_internal.hpp"
#include "refine_internal.hpp"

namespace nebem {

template <typename T>
static nebem_status lu_factor_checked(T *A, int n, int *ipiv, std::vector<int> &perm, hipStream_t st)
{
    const int nblk = (n + 255) / 256;
    DevBuf pval, ws, sync;
    NEBEM_HIP(pval.alloc((size_t)nblk * sizeof(T), st));
    NEBEM_HIP(ws.alloc((size_t)(nblk + 2) * sizeof(int), st));
    LUWork w;
    w.pval = pval.p;
    w.pidx = ws.as<int>();
    w.counter = ws.as<int>() + nblk;
    w.info = ws.as<int>() + nblk + 1;
    // single-launch panel scratch: bar, timeout | cidx (2 G) | cval (2 G) |
    // trow (2 kNB) | crow (2 G kNB), each part 256-byte aligned
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_cidx = 256, o_cval = o_cidx + up(2 * (size_t)nblk * sizeof(int));
    const size_t o_trow = o_cval + up(2 * (size_t)nblk * sizeof(T)), o_crow = o_trow + up(2 * (size_t)kNB * sizeof(T));
    const size_t sync_bytes = o_crow + 2 * (size_t)nblk * kNB * sizeof(T);
    NEBEM_HIP(sync.alloc(sync_bytes, st));
    char *sb = (char *)sync.p;
    w.bar = (unsigned *)sb;
    w.timeout = (int *)(sb + sizeof(unsigned));
    w.cidx = (int *)(sb + o_cidx);
    w.cval = sb + o_cval;
    w.trow = sb + o_trow;
    w.crow = sb + o_crow;
    int hinfo = n;
    NEBEM_HIP(hipMemsetAsync(w.counter, 0, sizeof(int), st));
    NEBEM_HIP(hipMemsetAsync(sb, 0, 256, st));
    NEBEM_HIP(hipMemcpyAsync(w.info, &hinfo, sizeof(int), hipMemcpyHostToDevice, st));
    lu_factor(A, n, ipiv, w, st);
    NEBEM_HIP(hipGetLastError());
    std::vector<int> hpiv(n);
    int htimeout = 0;
    NEBEM_HIP(hipMemcpyAsync(&hinfo, w.info, sizeof(int), hipMemcpyDeviceToHost, st));
    NEBEM_HIP(hipMemcpyAsync(&htimeout, w.timeout, sizeof(int), hipMemcpyDeviceToHost, st));
    NEBEM_HIP(hipMemcpyAsync(hpiv.data(), ipiv, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
    NEBEM_HIP(hipStreamSynchronize(st));
    if (htimeout) return fail(NEBEM_EDEVICE, "solve: a panel barrier wait timed out");
    if (hinfo < n) {
        char buf[96];
        std::snprintf(buf, sizeof buf, "solve: zero pivot in column %d", hinfo);
        return fail(NEBEM_ESINGULAR, buf);
    }
    pivots_to_perm(hpiv, perm);
    return NEBEM_OK;
}

nebem_status factor_fp64(double *A, int n, int *ipiv, std::vector<int> &perm_host, hipStream_t st)
{
    return lu_factor_checked<double>(A, n, ipiv, perm_host, st);
}

nebem_status factor_mixed(const double *A, int n, float *A32, double *s, int *ipiv, std::vector<int> &perm_host,
                          hipStream_t st)
{
    DevBuf part;
    const int nchunk = (n + kRowChunk - 1) / kRowChunk;
    NEBEM_HIP(part.alloc((size_t)n * nchunk * sizeof(double), st));
    row_scale(A, n, part.as<double>(), s, st);
    convert_scaled(A, s, n, A32, st);
    NEBEM_HIP(hipGetLastError());
    return lu_factor_checked<float>(A32, n, ipiv, perm_host, st);
}

nebem_status solve_fp64(const double *LU, int n, const int *perm, const double *B, int nrhs, double *X,
                        hipStream_t st)
{
    DevBuf work, xtmp;
    NEBEM_HIP(work.alloc((size_t)n * nrhs * sizeof(double), st));
    double *x = X;
    if (X == B) {
        NEBEM_HIP(xtmp.alloc((size_t)n * nrhs * sizeof(double), st));
        x = xtmp.as<double>();
    }
    lu_solve(LU, n, perm, B, x, work.as<double>(), nrhs, st);
    NEBEM_HIP(hipGetLastError());
    if (x != X) NEBEM_HIP(hipMemcpyAsync(X, x, (size_t)n * nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
    return NEBEM_OK;
}

static nebem_status host_norm(const double *sq_dev, int nblk, std::vector<double> &h, hipStream_t st, double &out)
{
    h.resize(nblk);
    NEBEM_HIP(hipMemcpyAsync(h.data(), sq_dev, (size_t)nblk * sizeof(double), hipMemcpyDeviceToHost, st));
    NEBEM_HIP(hipStreamSynchronize(st));
    double acc = 0.0;
    for (int k = 0; k < nblk; ++k) acc += h[k];
    out = std::sqrt(acc);
    return NEBEM_OK;
}

nebem_status refine_fp64(const double *A, const double *LU, const int *perm, int n, const double *b, double *x,
                         int max_steps, nebem_solve_info *info, hipStream_t st)
{
    const int nblk = (n + 255) / 256;
    const int nchunk = (n + kGemvChunk - 1) / kGemvChunk;
    DevBuf ones, rs, d, w, part, sq, xbest;
    NEBEM_HIP(ones.alloc((size_t)n * sizeof(double), st));
    NEBEM_HIP(rs.alloc((size_t)n * sizeof(double), st));
    NEBEM_HIP(d.alloc((size_t)n * sizeof(double), st));
    NEBEM_HIP(w.alloc((size_t)n * sizeof(double), st));
    NEBEM_HIP(part.alloc((size_t)n * nchunk * sizeof(double), st));
    NEBEM_HIP(sq.alloc((size_t)nblk * sizeof(double), st));
    NEBEM_HIP(xbest.alloc((size_t)n * sizeof(double), st));
    fill(ones.as<double>(), n, 1.0, st);
    std::vector<double> h;
    double bnorm = 0.0, rnorm = 0.0;
    sumsq(b, n, sq.as<double>(), st);
    nebem_status e = host_norm(sq.as<double>(), nblk, h, st, bnorm);
    if (e) return e;
    if (info) {
        info->ir_iters = 0;
        info->rel_resid = 0.0;
    }
    if (bnorm == 0.0) return NEBEM_OK;
    residual(A, n, x, b, ones.as<double>(), part.as<double>(), rs.as<double>(), sq.as<double>(), st);
    NEBEM_HIP(hipGetLastError());
    if ((e = host_norm(sq.as<double>(), nblk, h, st, rnorm))) return e;
    double best = rnorm / bnorm;
    int best_it = 0;
    NEBEM_HIP(hipMemcpyAsync(xbest.p, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int it = 1; it <= max_steps; ++it) {
        lu_solve(LU, n, perm, rs.as<double>(), d.as<double>(), w.as<double>(), 1, st);
        add_f64(x, d.as<double>(), n, st);
        residual(A, n, x, b, ones.as<double>(), part.as<double>(), rs.as<double>(), sq.as<double>(), st);
        NEBEM_HIP(hipGetLastError());
        if ((e = host_norm(sq.as<double>(), nblk, h, st, rnorm))) return e;
        const double rel = rnorm / bnorm;
        const bool halved = rel <= 0.5 * best;
        if (rel < best) {
            best = rel;
            best_it = it;
            NEBEM_HIP(hipMemcpyAsync(xbest.p, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
        if (!halved) break;
    }
    NEBEM_HIP(hipMemcpyAsync(x, xbest.p, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    NEBEM_HIP(hipStreamSynchronize(st));
    if (info) {
        info->ir_iters = best_it;
        info->rel_resid = best;
    }
    return NEBEM_OK;
}

nebem_status norm1_fp64(const double *A, int n, double *anorm, hipStream_t st)
{
    DevBuf cs;
    NEBEM_HIP(cs.alloc((size_t)n * sizeof(double), st));
    column_abs_sums(A, n, cs.as<double>(), st);
    NEBEM_HIP(hipGetLastError());
    std::vector<double> h(n);
    NEBEM_HIP(hipMemcpyAsync(h.data(), cs.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
    NEBEM_HIP(hipStreamSynchronize(st));
    double m = 0.0;
    for (int j = 0; j < n; ++j) m = h[j] > m ? h[j] : m;
    *anorm = m;
    return NEBEM_OK;
}

// ||A^-1||_1 by Hager's method (W. W. Hager, SIAM J. Sci. Stat. Comput.
// 5(2):311-316, 1984) with N. J. Higham's safeguards (ACM TOMS 14(4):
// 381-396, 1988): at most 5 sweeps x -> A^-1 x -> sign -> A^-T, stopping
// when the estimate stops growing or the gradient test fails, and the
// alternating test vector x_i = (-1)^i (1 + i/(n-1)).  A lower bound,
// usually within a factor 3 of the true norm.
nebem_status condest_fp64(const double *LU, const int *perm, int n, double anorm, double *kappa, hipStream_t st)
{
    DevBuf x, y, z, w, v;
    for (DevBuf *b : {&x, &y, &z, &w, &v}) NEBEM_HIP(b->alloc((size_t)n * sizeof(double), st));
    std::vector<double> hx(n, 1.0 / n), hy(n), hz(n), hs(n);
    auto solve = [&](const std::vector<double> &in, std::vector<double> &out, bool transposed) -> nebem_status {
        NEBEM_HIP(hipMemcpyAsync(x.p, in.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, st));
        if (transposed)
            lu_solve_transposed(LU, n, perm, x.as<double>(), y.as<double>(), w.as<double>(), v.as<double>(), st);
        else
            lu_solve(LU, n, perm, x.as<double>(), y.as<double>(), w.as<double>(), 1, st);
        NEBEM_HIP(hipGetLastError());
        NEBEM_HIP(hipMemcpyAsync(out.data(), y.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
        NEBEM_HIP(hipStreamSynchronize(st));
        return NEBEM_OK;
    };
    auto norm1 = [](const std::vector<double> &a) {
        double t = 0.0;
        for (double e : a) t += std::fabs(e);
        return t;
    };
    nebem_status e;
    double est = 0.0;
    int jlast = -1;
    for (int it = 0; it < 5; ++it) {
        if ((e = solve(hx, hy, false))) return e;
        const double ne = norm1(hy);
        if (it > 0 && ne <= est) break;
        est = ne;
        for (int i = 0; i < n; ++i) hs[i] = hy[i] >= 0.0 ? 1.0 : -1.0;
        if ((e = solve(hs, hz, true))) return e;
        int j = 0;
        double zx = 0.0;
        for (int i = 0; i < n; ++i) {
            if (std::fabs(hz[i]) > std::fabs(hz[j])) j = i;
            zx += hz[i] * hx[i];
        }
        if (it > 0 && (j == jlast || std::fabs(hz[j]) <= zx)) break;
        jlast = j;
        std::fill(hx.begin(), hx.end(), 0.0);
        hx[j] = 1.0;
    }
    for (int i = 0; i < n; ++i) hx[i] = (i & 1 ? -1.0 : 1.0) * (1.0 + (n > 1 ? (double)i / (n - 1) : 0.0));
    if ((e = solve(hx, hy, false))) return e;
    const double alt = 2.0 * norm1(hy) / (3.0 * n);
    *kappa = anorm * (alt > est ? alt : est);
    return NEBEM_OK;
}

nebem_status solve_mixed(const double *A, const float *LU32, const double *s, const int *perm, int n, const double *b,
                         double *x, double tol, int max_iter, nebem_solve_info *info, hipStream_t st)
{
    const int nblk = (n + 255) / 256;
    const int nchunk = (n + kGemvChunk - 1) / kGemvChunk;
    DevBuf rs, d32, w32, part, sq, xbest;
    NEBEM_HIP(rs.alloc((size_t)n * sizeof(double), st));
    NEBEM_HIP(d32.alloc((size_t)n * sizeof(float), st));
    NEBEM_HIP(w32.alloc((size_t)n * sizeof(float), st));
    NEBEM_HIP(part.alloc((size_t)n * nchunk * sizeof(double), st));
    NEBEM_HIP(sq.alloc((size_t)nblk * sizeof(double), st));
    NEBEM_HIP(xbest.alloc((size_t)n * sizeof(double), st));
    std::vector<double> h;
    double bnorm = 0.0;
    sumsq(b, n, sq.as<double>(), st);
    nebem_status e = host_norm(sq.as<double>(), nblk, h, st, bnorm);
    if (e) return e;
    fill(x, n, 0.0, st);
    if (info) {
        info->ir_iters = 0;
        info->rel_resid = 0.0;
    }
    if (bnorm == 0.0) return NEBEM_OK;
    scale_vec(s, b, n, rs.as<double>(), st);
    double best = INFINITY;
    int stall = 0, it = 0;
    for (it = 1; it <= max_iter; ++it) {
        lu_solve(LU32, n, perm, rs.as<double>(), d32.as<float>(), w32.as<float>(), 1, st);
        add_f32(x, d32.as<float>(), n, st);
        residual(A, n, x, b, s, part.as<double>(), rs.as<double>(), sq.as<double>(), st);
        NEBEM_HIP(hipGetLastError());
        double rnorm = 0.0;
        if ((e = host_norm(sq.as<double>(), nblk, h, st, rnorm))) return e;
        const double rel = rnorm / bnorm;
        if (rel < best) {
            stall = (rel > 0.5 * best) ? stall + 1 : 0;
            best = rel;
            NEBEM_HIP(hipMemcpyAsync(xbest.p, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
            if (info) {
                info->ir_iters = it;
                info->rel_resid = rel;
            }
        } else {
            ++stall;
        }
        if (best <= tol || stall >= 3) break;
    }
    if (best < INFINITY)  // otherwise no step was taken and x is still 0
        NEBEM_HIP(hipMemcpyAsync(x, xbest.p, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    NEBEM_HIP(hipStreamSynchronize(st));
    if (best <= tol) return NEBEM_OK;
    char buf[128];
    std::snprintf(buf, sizeof buf, "solve: refinement stopped at relative residual %.3e (tolerance %.1e)", best, tol);
    return fail(NEBEM_ENOCONV, buf);
}

}  // namespace nebem
