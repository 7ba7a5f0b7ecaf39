// charge_internal.hpp -- launchers of the point-charge kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nebem {

// ex/ey/ez += k_e sum_{j != i} q_j (x_i - x_j) / |x_i - x_j|^3 (coincident
// charges add nothing), over the charges in Morton order; ws of
// coulomb_workspace(nq) bytes (0 on error)
size_t coulomb_workspace(int64_t nq);
hipError_t launch_coulomb(const double *qx, const double *qy, const double *qz, const double *q, int64_t nq,
                          double *ex, double *ey, double *ez, void *ws, size_t ws_bytes, hipStream_t s);
// phi/ex/ey/ez (each may be null) += the field of nq point charges at m
// targets (FP32 pair terms, FP64 sums; coincident points add nothing)
void launch_point_field(const double *tx, const double *ty, const double *tz, int64_t m, const double *qx,
                        const double *qy, const double *qz, const double *q, int64_t nq, double *phi, double *ex,
                        double *ey, double *ez, hipStream_t s);
// partial sums of |q| into part[0 .. returned count) (<= kAbsParts); their
// sum in index order is sum_i |q_i|
constexpr int kAbsParts = 256;
int launch_abs_sum(const double *q, int64_t nq, double *part, hipStream_t s);
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
