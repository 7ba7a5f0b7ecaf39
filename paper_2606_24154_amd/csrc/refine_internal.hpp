// refine_internal.hpp -- launchers for the mixed-precision solve helpers.
#pragma once
#include <hip/hip_runtime.h>

namespace nebem {

constexpr int kRowChunk = 1024;   // columns per row-maximum partial
constexpr int kGemvChunk = 2048;  // columns per residual partial

// s[i] = 1 / max_j |A_ij| (1 for an all-zero row); part: n * ceil(n/kRowChunk) doubles
void row_scale(const double *A, int n, double *part, double *s, hipStream_t st);
// A32 = float(diag(s) A), column-major
void convert_scaled(const double *A, const double *s, int n, float *A32, hipStream_t st);
// rs = s .* (b - A x) in FP64; sq[k] = per-workgroup sums of (b - A x)^2 (ceil(n/256) entries);
// part: n * ceil(n/kGemvChunk) doubles
void residual(const double *A, int n, const double *x, const double *b, const double *s, double *part, double *rs,
              double *sq, hipStream_t st);
void sumsq(const double *v, int n, double *sq, hipStream_t st);
void add_f32(double *x, const float *d, int n, hipStream_t st);
void add_f64(double *x, const double *d, int n, hipStream_t st);
// cs[j] = sum_i |A_ij|, n entries
void column_abs_sums(const double *A, int n, double *cs, hipStream_t st);
void scale_vec(const double *s, const double *b, int n, double *out, hipStream_t st);
void fill(double *x, int n, double v, hipStream_t st);

}  // namespace nebem
