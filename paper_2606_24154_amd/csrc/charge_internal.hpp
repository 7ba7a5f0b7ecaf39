// charge_internal.hpp -- launchers of the point-charge kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nebem {

// ex/ey/ez += k_e sum_{j != i} q_j (x_i - x_j) / |x_i - x_j|^3 (coincident charges skipped)
void launch_coulomb_self(const double *qx, const double *qy, const double *qz, const double *q, int64_t nq, double *ex,
                         double *ey, double *ez, hipStream_t s);
// number of source chunks for launch_charge_rhs (part holds nchunk * n doubles)
int charge_rhs_chunks(int64_t n, int64_t nq);
// b = b0 - (phi_q(c_i) on conductor rows, n_i . E_q(c_i) on dielectric rows)
void launch_charge_rhs(const double *drec, int64_t n, const double *qx, const double *qy, const double *qz,
                       const double *q, int64_t nq, const double *b0, double *part, int nchunk, double *b,
                       hipStream_t s);
// x += sign(q) mu_dt E
void launch_euler(double *qx, double *qy, double *qz, const double *q, const double *ex, const double *ey,
                  const double *ez, int64_t nq, double mu_dt, hipStream_t s);
void launch_boundary_values(const int *bc, const double *value, int64_t n, double *b0, hipStream_t s);

}  // namespace nebem
