// host_util.hpp -- host-side helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "nebem_internal.hpp"

namespace nebem {

// Stream-ordered device buffer owned by one call (or one session).
struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFreeAsync(p, s);
        p = nullptr;
    }
    hipError_t alloc(size_t bytes, hipStream_t stream)
    {
        release();
        s = stream;
        return hipMallocAsync(&p, bytes ? bytes : 8, stream);
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

nebem_status check_panels(const nebem_panels *p);
// Validated voxel grid of the point-to-line reduction (>= 1 voxel per axis,
// fewer than 2^32 - 1 in all)
nebem_status voxel_grid_args(const nebem_grid *vox, GridArgs &g);
nebem_status check_options(const nebem_options &o);
// Derived element records (validated; synchronises the stream).
nebem_status derive(const nebem_panels *p, hipStream_t s, DevBuf &drec);
// run_eval with a stream-ordered workspace of its preferred size (api.hip)
nebem_status eval_with_workspace(const double *drec, const double *sigma, int64_t n, int ncol, const ImgArgs &ia,
                                 int mixed, double near_factor, const double *px, const double *py, const double *pz,
                                 int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t stream,
                                 const char *what);
void pivots_to_perm(const std::vector<int> &ipiv, std::vector<int> &perm);

// Dense solve drivers (solver.hip).  FP64: A is factored in place.
// MIXED: A untouched; A32 (n*n floats), scale s (n) and perm/ipiv receive the
// equilibrated FP32 factorisation.
nebem_status factor_fp64(double *A, int n, int *ipiv, std::vector<int> &perm_host, hipStream_t st);
nebem_status factor_mixed(const double *A, int n, float *A32, double *s, int *ipiv, std::vector<int> &perm_host,
                          hipStream_t st);
// X = A^-1 B for nrhs columns with FP64 factors (perm on device)
nebem_status solve_fp64(const double *LU, int n, const int *perm, const double *B, int nrhs, double *X,
                        hipStream_t st);
// FP64 refinement of an FP64 LU solution x (one column), against the
// unfactored A: r = b - A x, x += LU^-1 r while ||r|| at least halves, at most
// max_steps steps; x ends as the iterate with the smallest residual.
nebem_status refine_fp64(const double *A, const double *LU, const int *perm, int n, const double *b, double *x,
                         int max_steps, nebem_solve_info *info, hipStream_t st);
constexpr int kFp64RefineSteps = 3;
// ||A||_1 (host result) and the 1-norm condition estimate anorm x est(||A^-1||_1)
// from FP64 factors (Hager-Higham); both synchronise the stream.
nebem_status norm1_fp64(const double *A, int n, double *anorm, hipStream_t st);
nebem_status condest_fp64(const double *LU, const int *perm, int n, double anorm, double *kappa, hipStream_t st);
// refinement: x solves A x = b to ||b - A x|| <= tol ||b||, one column
nebem_status solve_mixed(const double *A, const float *LU32, const double *s, const int *perm, int n, const double *b,
                         double *x, double tol, int max_iter, nebem_solve_info *info, hipStream_t st);

}  // namespace nebem
