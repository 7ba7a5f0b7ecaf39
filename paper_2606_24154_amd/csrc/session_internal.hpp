// session_internal.hpp -- the resident-geometry object behind nebem_session.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "nebem_internal.hpp"

namespace nebem {

// plain device allocation owned by a session (freed with the session)
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t ensure(size_t b)
    {
        if (b <= bytes && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, b ? b : 8);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

}  // namespace nebem

struct nebem_session {
    int64_t n = 0;
    double img_count = 1.0;  // copies per element (reflections x translations)
    nebem_options opt;
    nebem::ImgArgs img;
    nebem::DevMem drec, A, LU, A32, scale, ipiv, perm, b0, sigma, rhs, part, eb;
    nebem::DevMem lines, lf, vws;  // line charges, their field at the charges, the reduction's workspace
    nebem::DevMem ows;  // workspace of the Morton-ordered evaluation
    nebem::DevMem cws;  // workspace of the charge-pair sums (Morton order of the charges)
    nebem_solve_info last_info = {0, -1.0};
    // FastVolume map regenerated after every space-charge re-solve
    int fv_kind = 0;  // 0 none, 1 regular grid, 2 graded axes
    nebem::GridArgs fv_grid = {};
    nebem::AxesArgs fv_axes = {};
    double *fv_values = nullptr;  // caller's buffer, 4 doubles per node
    int64_t fv_nodes = 0;
    nebem::DevMem fv_tmp;  // nodes (3) and field (4) columns
    nebem::DevMem absq;    // partial sums of |q| (threshold rule)
};
