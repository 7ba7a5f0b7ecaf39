// lu_internal.hpp -- dense LU factorisation / solve launchers.
#pragma once
#include <hip/hip_runtime.h>

namespace nebem {

constexpr int kNB = 64;        // LU panel width
constexpr int kOuterNB = 256;  // LU outer block width (multiple of kNB)

// Device scratch of one factorisation: per-workgroup pivot candidates
// (ceil(n/256) entries), a completion counter (must start at 0; every panel
// launch leaves it at 0) and `info` (must start at n; receives the first
// column with a zero pivot).
// The single-launch panel factorisation (taken when cval is not null and
// the panel's workgroups fit on the device at once) also needs, with
// G = ceil(n/256): cval 2 G entries of the matrix type, cidx 2 G ints, crow
// 2 G kNB entries, trow 2 kNB entries, a barrier counter `bar` and a flag
// `timeout`, both starting at 0; `timeout` is set if a barrier wait gave up.
struct LUWork {
    void *pval;
    int *pidx;
    int *counter;
    int *info;
    void *cval = nullptr;
    int *cidx = nullptr;
    void *crow = nullptr;
    void *trow = nullptr;
    unsigned *bar = nullptr;
    int *timeout = nullptr;
};

void lu_factor(double *A, int n, int *ipiv, LUWork &w, hipStream_t s);
void lu_factor(float *A, int n, int *ipiv, LUWork &w, hipStream_t s);
// X = A^-1 B with the row permutation perm (X[i] = (P B)[i] = B[perm[i]]);
// W is an n x nrhs workspace of the solve's type.
void lu_solve(const double *LU, int n, const int *perm, const double *B, double *X, double *W, int nrhs,
              hipStream_t s);
void lu_solve(const float *LU, int n, const int *perm, const double *B, float *X, float *W, int nrhs,
              hipStream_t s);
// z = A^-T b with the FP64 factors of P A = L U (perm as in lu_solve); W, V:
// n-entry workspaces.  z must not alias b, W or V.
void lu_solve_transposed(const double *LU, int n, const int *perm, const double *b, double *z, double *W,
                         double *V, hipStream_t s);

}  // namespace nebem
