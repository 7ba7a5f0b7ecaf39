/*
 * nebem.h -- C-ABI of libnebem, the MI355X (gfx950) hot path of the nearly
 * exact boundary element method (neBEM) for electrostatics.
 *
 * The method (paper: "neBEM: A GPU-accelerated Electrostatic Field Solver"):
 *  - boundaries are cut into flat rectangular and right-triangular elements
 *    carrying a uniform surface charge density (Sec. 2, zeroth-order BEM);
 *  - the potential and field of each element are its exact closed-form
 *    integrals of the free-space Green's function (Sec. 2.1);
 *  - collocation at element centroids gives K sigma = phi (Eq. Matrix),
 *    solved for sigma (Algorithm 1, LU factorisation);
 *  - potential and field anywhere follow by superposition over all
 *    elements and their periodic copies (Eqs. Potential and Field; Sec. 3,
 *    PFAtPoint in Sec. 4.1), plus known point charges (Sec. 4.2, Algorithm 2);
 *  - the dynamic space-charge loop moves charges and re-solves sigma with the
 *    charges on the right-hand side (Sec. 4.3, Algorithm 4).
 *
 * Conventions for every entry point
 *  - SI units: metres, volts, coulombs, C/m^2, V/m.
 *  - Every array argument is DEVICE memory on the current HIP device, owned
 *    by the caller, unless marked "host".  Arrays are structure-of-arrays,
 *    contiguous, FP64 unless stated.  Matrices are column-major with leading
 *    dimension n.
 *  - Work is enqueued on `stream`; outputs are valid after the stream has
 *    synchronised.  Calls that need a host decision (pivot failure, solver
 *    convergence, panel validation) synchronise `stream` themselves and say so.
 *  - Return value 0 = NEBEM_OK, negative = error; nebem_last_error() gives a
 *    thread-local message.  Validation errors return before any kernel
 *    launch that writes caller memory.  No C++ exception crosses this ABI.
 *  - The library keeps no state between calls except inside nebem_session
 *    objects.  Stateless calls allocate their temporaries stream-ordered
 *    (hipMallocAsync / hipFreeAsync on `stream`).
 */
#ifndef NEBEM_H
#define NEBEM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nebem_status;
#define NEBEM_OK 0
#define NEBEM_EINVAL (-1)    /* bad argument or invalid panel */
#define NEBEM_ENOMEM (-2)    /* device allocation failed */
#define NEBEM_ESINGULAR (-3) /* exactly zero pivot in the LU factorisation */
#define NEBEM_ENOCONV (-4)   /* iterative refinement did not reach ir_tol */
#define NEBEM_EDEVICE (-5)   /* HIP runtime error */
#define NEBEM_EBUSY (-6)     /* serving queue full / request exceeds budget */

/* Element kinds (Sec. 2.1: rectangular and right-angled triangular elements) */
#define NEBEM_RECT 0 /* { o + s u + t w : 0 <= s,t <= 1 } */
#define NEBEM_RTRI 1 /* { o + s u + t w : s,t >= 0, s + t <= 1 }, right angle at o */

/* Boundary conditions (Sec. 2: Dirichlet on conductors; dielectric interfaces
 * are a reading -- continuity of the normal displacement, see nebem_assemble) */
#define NEBEM_CONDUCTOR 0
#define NEBEM_DIELECTRIC 1

/* Panels, structure of arrays, n entries each.  u and w must be perpendicular
 * (|u.w| <= 1e-9 |u||w|) and non-zero; the unit normal is n = u x w / |u x w|.
 * eps_pos / eps_neg: relative permittivity on the +n / -n side (only read for
 * dielectric panels).  value: conductor potential (only read where needed). */
typedef struct nebem_panels {
    int64_t n;
    const int32_t *kind;
    const double *ox, *oy, *oz;
    const double *ux, *uy, *uz;
    const double *wx, *wy, *wz;
    const int32_t *bc;
    const double *value;
    const double *eps_pos, *eps_neg;
} nebem_panels;

/* Copies of the base cell (host struct, passed by pointer, copied by the call).
 * Translations t = i a1 + j a2, -n1 <= i <= n1, -n2 <= j <= n2 (Sec. 3 and
 * Sec. 5.2: "virtual copies" of a base cell).  Optional reflection planes
 * x_k = mirror_pos[k] for each axis bit k (1 = x, 2 = y, 4 = z) in
 * mirror_mask; a copy reflected in a set of planes carries sigma times the
 * product of their mirror_parity (+1/-1).  copy = t + M(panel).  Every copy
 * enters both assembly and evaluation; known point charges are not copied.
 * n1, n2 <= 64. */
typedef struct nebem_images {
    double a1[3], a2[3];
    int32_t n1, n2;
    int32_t mirror_mask;
    double mirror_pos[3];
    int32_t mirror_parity[3];
} nebem_images;

typedef enum nebem_precision {
    NEBEM_FP64 = 0,  /* exact closed forms in FP64 everywhere; FP64 LU + FP64 refinement */
    NEBEM_MIXED = 1  /* FP64 near field, FP64 monopole + FP32 correction far away; FP32 LU + FP64 refinement */
} nebem_precision;

typedef struct nebem_options {
    int32_t precision;     /* nebem_precision */
    double near_factor;    /* mixed: exact FP64 at least for R < near_factor * D (default 4); the FP32
                              corrections start at max(near_factor, 24) D for rectangles and
                              max(near_factor, 48) D for triangles (R from the centroid, D = diameter) */
    double ir_tol;         /* mixed solve: stop at ||b - A x||_2 / ||b||_2 <= ir_tol (1e-10) */
    int32_t ir_max_iter;   /* mixed solve: refinement steps (30) */
    double sc_dt;          /* space charge: time step, s (1e-12) */
    double sc_mobility;    /* space charge: |v| = mobility |E|, m^2/(V s) (1e-4) */
    int32_t sc_resolve_every; /* space charge: re-solve sigma every k steps (10), when sc_threshold < 0 */
    double sc_threshold;   /* space charge (Algorithm 4's SpChTh): >= 0: re-solve at a step when the
                              charges' magnitude sum_i |q_i| exceeds it, C, checked every step; < 0
                              (default -1): the fixed schedule sc_resolve_every */
} nebem_options;

typedef struct nebem_solve_info {
    int32_t ir_iters;     /* refinement steps taken (worst column) */
    double rel_resid;     /* ||b - A x||_2 / ||b||_2 of the returned x, FP64 (worst column; -1 if not computed) */
} nebem_solve_info;

/* Fills `opt` with the defaults listed above. */
void nebem_default_options(nebem_options *opt);

/* Influence matrix (Eq. Matrix; collocation at centroids, Sec. 2).  Row i is
 * the collocation point c_i (cx/cy/cz, n entries each, or all three NULL for
 * the panel centroids); column j the unit-density panel j with all its
 * copies.  With k_e = 1/(4 pi eps0):
 *   conductor row:  A_ij = k_e sum_copies Phi'_j(c_i)
 *   dielectric row: A_ij = k_e sum_copies n_i . E'_j(c_i)
 *                          + [i == j] (eps+ + eps-) / (2 eps0 (eps+ - eps-))
 * where Phi', E' are the exact potential and field integrals of Sec. 2.1,
 * in both precision modes (opt->precision does not change the matrix).
 * Panel i's own (untranslated, unreflected) copy is evaluated with c_i taken
 * exactly in its plane (principal value of the normal field = 0).
 * A: n x n FP64, column-major, caller-allocated (8 n^2 bytes). */
nebem_status nebem_assemble(const nebem_panels *panels, const nebem_images *images, const double *cx,
                            const double *cy, const double *cz, const nebem_options *opt, double *A,
                            hipStream_t stream);

/* Solves A sigma = b for nrhs right-hand sides (Eq. Matrix; Algorithm 1's LU
 * factorisation with row pivoting, without forming the inverse).
 *  FP64 mode: A (n x n, column-major) is overwritten by its LU factors
 *    (unit lower L below the diagonal, U on and above), ipiv[k] (int32, n
 *    entries, 0-based) is the row swapped with row k at step k.  The LU
 *    solution is then refined in FP64 (r = b - A x against a temporary copy
 *    of the unfactored A, x += LU^-1 r) while each step at least halves
 *    ||r||, at most 3 steps (fixed-precision refinement: on the double
 *    THGEM, N = 41 600, the relative residual goes from 5.1e-12 to 4.2e-13
 *    in one step and sigma moves by 1.4e-9 relative).  If the n x n copy
 *    cannot be allocated, the LU solution is returned unrefined
 *    (info->ir_iters 0, rel_resid -1).
 *  MIXED mode: A is left unchanged; the library factors an FP32 copy and
 *    refines in FP64 until ||b - A x||_2 <= ir_tol ||b||_2 per column.
 *    ipiv holds the FP32 factorisation's pivots.
 * b, sigma: n x nrhs column-major (may alias).  `info` (host, may be NULL)
 * receives iteration count and residual.  Synchronises `stream`.
 * Returns NEBEM_ESINGULAR on an exactly zero pivot, NEBEM_ENOCONV if
 * refinement stalls (sigma then holds the best iterate). */
nebem_status nebem_solve(double *A, int64_t n, const double *b, int64_t nrhs, double *sigma, int32_t *ipiv,
                         const nebem_options *opt, nebem_solve_info *info, hipStream_t stream);

/* Re-solves with factors from a previous FP64-mode nebem_solve (the paper
 * keeps the factorised matrix resident for new right-hand sides, Sec. 4.1). */
nebem_status nebem_solve_factored(const double *LU, const int32_t *ipiv, int64_t n, const double *b,
                                  int64_t nrhs, double *sigma, hipStream_t stream);

/* Conditioning of the dense system.  nebem_norm1: ||A||_1 = max_j sum_i |A_ij|
 * of the column-major n x n matrix A (device), written to *anorm (host).
 * nebem_condest: 1-norm condition estimate anorm * est(||A^-1||_1) from the
 * FP64 factors and pivots of nebem_solve (LAPACK gecon's estimator: Hager's
 * method with Higham's safeguards, at most 5 pairs of solves with A and A^T
 * plus one; a lower bound on cond_1(A), usually within a factor 3), written
 * to *kappa1 (host).  anorm is ||A||_1 of the unfactored matrix (take it
 * with nebem_norm1 before nebem_solve overwrites A).  Both synchronise
 * `stream`.  EINVAL on bad sizes, NULL pointers, an invalid pivot list or a
 * negative anorm. */
nebem_status nebem_norm1(const double *A, int64_t n, double *anorm, hipStream_t stream);
nebem_status nebem_condest(const double *LU, const int32_t *ipiv, int64_t n, double anorm, double *kappa1,
                           hipStream_t stream);

/* Potential and field at m points (Eqs. Potential and Field; PFAtPoint,
 * Sec. 4.1) from all panels and their copies:
 *   phi(P) = k_e sum_j sigma_j sum_copies Phi'_j(P),  E likewise with E'.
 * px/py/pz: m points; phi/ex/ey/ez: m outputs (any of the four may be NULL
 * to skip storing it).  sigma: n densities (C/m^2). */
nebem_status nebem_eval(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                        const double *px, const double *py, const double *pz, int64_t m, double *phi,
                        double *ex, double *ey, double *ez, const nebem_options *opt, hipStream_t stream);

/* Weighting fields (Sec. 2.1: one readout at unit potential, the others at
 * zero, one sigma per readout): phi and E at m points for nsig density
 * columns at once.  sigma: n x nsig column-major (column k at sigma + k n);
 * phi/ex/ey/ez: m x nsig column-major (column k at phi + k m), any of the
 * four may be NULL.  The element copies' closed forms are evaluated once per
 * point for up to 4 columns (larger nsig is done 4 columns at a time), so
 * the transcendentals are shared between readouts; column k equals
 * nebem_eval with that column bit for bit.  nsig <= 64.  Other arguments as
 * in nebem_eval. */
nebem_status nebem_eval_multi(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                              int64_t nsig, const double *px, const double *py, const double *pz, int64_t m,
                              double *phi, double *ex, double *ey, double *ez, const nebem_options *opt,
                              hipStream_t stream);

/* Adaptive Modelling (Sec. 3: far away, a periodic structure's fine charge
 * distribution is replaced by the average density of each primitive).
 * `prims` are the primitives the elements were cut from (flat rectangles /
 * right triangles, same layout as `panels`; bc/value/eps are not read),
 * elem_prim[j] (device, n entries) the primitive of element j.  Translated
 * copies with |i1| <= prim_after and |i2| <= prim_after (with every
 * reflection) are summed element by element exactly as in nebem_eval; every
 * farther copy is summed primitive by primitive, each primitive with the
 * uniform density sigma_p = sum_{j in p} sigma_j A_j / A_p (the same total
 * charge) and the exact closed form of its own shape.  prim_after < 0: no
 * simplification (= nebem_eval).  Other arguments as in nebem_eval.
 * Synchronises `stream`. */
nebem_status nebem_eval_adaptive(const nebem_panels *panels, const nebem_panels *prims, const int32_t *elem_prim,
                                 int32_t prim_after, const nebem_images *images, const double *sigma, const double *px,
                                 const double *py, const double *pz, int64_t m, double *phi, double *ex, double *ey,
                                 double *ez, const nebem_options *opt, hipStream_t stream);

/* FastVolume (Sec. 3: a volume sampled once on a regular grid, then
 * interpolated).  Grid nodes origin + (i step[0], j step[1], k step[2]),
 * 0 <= i < n[0] etc., each n >= 2, each step > 0; node (i, j, k) has index
 * q = i + n[0] (j + n[1] k).  Node values are interleaved: values[4 q + c]
 * with c = 0 phi, 1 ex, 2 ey, 3 ez (device, 4 n[0] n[1] n[2] doubles,
 * 16-byte aligned), so one interpolation gathers 8 corners x 32 bytes. */
typedef struct nebem_grid {
    double origin[3];
    double step[3];
    int32_t n[3];
} nebem_grid;

/* Fills `values` with phi and E at every grid node (one nebem_eval over the
 * nodes, node x = origin[0] + i * step[0] with the product and the sum each
 * rounded to FP64, likewise y, z; other arguments as in nebem_eval).
 * n[0] n[1] n[2] <= 2^31 - 257. */
nebem_status nebem_fastvol_build(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                                 const nebem_grid *grid, double *values, const nebem_options *opt,
                                 hipStream_t stream);

/* Trilinear interpolation of the node values at m points (px/py/pz device,
 * m each); phi/ex/ey/ez: m outputs, any may be NULL.  On each axis the cell
 * is floor((x - origin)/step) limited to [0, n - 2] and the weights are the
 * fractional distances to its faces.  A point outside the grid (a
 * coordinate below the first or above the last node, or NaN) gets NaN in
 * every output, so the caller can evaluate it directly instead. */
nebem_status nebem_fastvol_interp(const nebem_grid *grid, const double *values, const double *px, const double *py,
                                  const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                                  hipStream_t stream);

/* Graded FastVolume grid: node (i, j, k) at (x[i], y[j], z[k]), each axis
 * a strictly increasing array of finite coordinates (device memory, caller
 * owned, n >= 2 per axis, n[0] n[1] n[2] <= 2^31 - 257), so that nodes can
 * be dense where the field varies fast (near electrodes and holes) and
 * sparse elsewhere.  Node index and value layout as for nebem_grid. */
typedef struct nebem_axes {
    const double *x, *y, *z;
    int32_t n[3];
} nebem_axes;

/* phi and E at every node of a graded grid (one nebem_eval over the nodes);
 * EINVAL if an axis is not strictly increasing and finite (checked on the
 * device before the evaluation; synchronises `stream`). */
nebem_status nebem_fastvol_build_axes(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                                      const nebem_axes *grid, double *values, const nebem_options *opt,
                                      hipStream_t stream);

/* Trilinear interpolation on a graded grid: per axis the cell is the last
 * node at or below the coordinate (binary search; the last cell for the
 * last node), the weights the fractional position in it; points outside
 * [first node, last node] on any axis get NaN.  Axes as given to the build
 * (not re-checked here: with axes that are not increasing the results are
 * meaningless but every read stays inside the arrays). */
nebem_status nebem_fastvol_interp_axes(const nebem_axes *grid, const double *values, const double *px,
                                       const double *py, const double *pz, int64_t m, double *phi, double *ex,
                                       double *ey, double *ez, hipStream_t stream);

/* Point charges reduced to line charges (Algorithm 3, voxelisation): the
 * charges are binned into the voxels of `vox` (voxel (i, j, k) =
 * floor((x - origin) / step) per axis, 1 <= n, n[0] n[1] n[2] < 2^32 - 1;
 * charges outside are dropped and counted in *outside, host, may be NULL);
 * every occupied voxel becomes one segment parallel to z over the voxel's
 * z extent, with line density = total charge / dz, placed in x, y by
 * `placement`: NEBEM_LINE_CENTRE through the voxel's centre (Algorithm 3's
 * voxel record holds only the total charge and the occupancy), or
 * NEBEM_LINE_WEIGHTED at the |q|-weighted mean x, y of its charges (the
 * centre if those weights sum to zero; a lone charge's line then passes
 * exactly through it); any other value is EINVAL.
 * lines: 7 doubles per line (ax, ay, az, bx, by, bz, lambda), device,
 * max_lines of them; *nlines (host) receives the number of occupied voxels,
 * lines in increasing voxel index.  EINVAL when *nlines > max_lines
 * (nothing written; call again with room for *nlines).  Deterministic: the
 * charges are sorted by voxel (stable) instead of accumulated with atomics.
 * Allocates a stream-ordered workspace of ~36 B per charge; synchronises
 * `stream`. */
enum { NEBEM_LINE_CENTRE = 0, NEBEM_LINE_WEIGHTED = 1 };
nebem_status nebem_voxelize_charges(const double *qx, const double *qy, const double *qz, const double *q,
                                    int64_t nq, const nebem_grid *vox, int32_t placement, double *lines,
                                    int64_t max_lines, int64_t *nlines, int64_t *outside, hipStream_t stream);

/* The charges' own field at every charge with the charges reduced to line
 * charges (Algorithm 3 as the source of the space-charge field, Sec. 4.2):
 * at a charge in voxel (i, j, k), the lines of all voxels outside
 * (i +- 1, j +- 1, k +- 1) plus the charges of those 27 voxels one by one
 * (k_e q (x - x_j)/|x - x_j|^3, FP32 per pair with FP64 sums of up to 64
 * pairs, coincident charges skipped), so no charge feels the line that
 * contains it; a charge outside the grid feels every line.  ex/ey/ez
 * (device, nq each) are overwritten; *nlines (may be NULL) receives the
 * number of lines.  Grid, placement and workspace as in
 * nebem_voxelize_charges; synchronises `stream`. */
nebem_status nebem_charge_field_lines(const double *qx, const double *qy, const double *qz, const double *q,
                                      int64_t nq, const nebem_grid *vox, int32_t placement, double *ex, double *ey,
                                      double *ez, int64_t *nlines, hipStream_t stream);

/* phi and E (k_e lambda times the exact segment integrals) of nlines
 * uniformly charged segments (layout as above) at m points; outputs as in
 * nebem_eval.  A point on a segment gets infinite phi and the principal
 * value 0 for the field across the segment; at a segment's end the results
 * are not finite.  A segment of zero length contributes nothing. */
nebem_status nebem_line_field(const double *lines, int64_t nlines, const double *px, const double *py,
                              const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                              hipStream_t stream);

/* ---------------------------------------------------------------- sessions
 * A session keeps one geometry resident: derived panel data, its influence
 * matrix and factors (FP64: the matrix and its FP64 LU, 16 n^2 bytes, every
 * solve refined as in nebem_solve; MIXED: the matrix and the FP32 LU,
 * 12 n^2 bytes), the boundary values and the current sigma (Sec. 4.1: the
 * factorised matrix stays in device memory for new right-hand sides). */
typedef struct nebem_session nebem_session;

/* Builds the derived element records, assembles and factors A (precision
 * per opt), solves for the panels' own boundary values (V on conductors, 0 on
 * dielectric interfaces).  The panel arrays are not referenced after the
 * call.  Synchronises `stream`.  Returns NEBEM_ENOCONV together with a usable
 * session if the mixed-precision refinement of that first solve stalled. */
nebem_status nebem_session_create(const nebem_panels *panels, const nebem_images *images,
                                  const nebem_options *opt, hipStream_t stream, nebem_session **out);
void nebem_session_destroy(nebem_session *s);
int64_t nebem_session_n(const nebem_session *s);
/* Device pointer to the session's current sigma (n entries, read-only). */
const double *nebem_session_sigma(const nebem_session *s);
/* Replaces the session's sigma by A^-1 b for a new right-hand side b (n
 * entries), e.g. a weighting-field set-up: unit potential on one readout,
 * zero elsewhere (Sec. 2.1).  `info` (host, may be NULL) as in nebem_solve.
 * Synchronises `stream`. */
nebem_status nebem_session_solve(nebem_session *s, const double *b, nebem_solve_info *info, hipStream_t stream);
/* cond_1 estimate of an FP64 session's matrix (as nebem_condest, from the
 * session's matrix and factors), written to *kappa1 (host).  EINVAL for a
 * MIXED session.  Synchronises `stream`. */
nebem_status nebem_session_condest(nebem_session *s, double *kappa1, hipStream_t stream);
/* phi/E at points with the session's current sigma (as nebem_eval). */
nebem_status nebem_session_eval(nebem_session *s, const double *px, const double *py, const double *pz,
                                int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t stream);

/* nebem_session_eval for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same results, bit for bit, with no allocation.  The
 * evaluation's workspace (element-segment partial sums, the Morton sort of
 * the points) lives in a fixed 64 MiB scratch array in device memory, one
 * per GPU, that the library holds until the process ends; points are taken
 * in chunks that fit it.  Every call on a GPU uses that GPU's one scratch:
 * calls that overlap on one GPU (other host threads, other streams) race
 * and must be serialised by the caller.  EINVAL when even a 256-point chunk
 * of this session's evaluation would not fit (more element segments than
 * the scratch allows) or m is out of range. */
nebem_status nebem_session_eval_noalloc(nebem_session *s, const double *px, const double *py, const double *pz,
                                        int64_t m, double *phi, double *ex, double *ey, double *ez,
                                        hipStream_t stream);

/* FastVolume map kept by the session (Algorithm 4's CreateFastVolPF): with
 * exactly one of `grid` (regular) or `axes` (graded) given, the session
 * fills `values` (device, caller owned, 4 doubles per node as in
 * nebem_fastvol_build, 16-byte aligned, kept alive by the caller, as are
 * graded axes) with phi and E at the nodes now, and again after every
 * re-solve of a space-charge step, then with the panels' field plus the
 * charges' own field at the nodes (the point charges, or the lines of a
 * nebem_spacecharge_step_lines step) at the step's start-of-step
 * positions.  Both NULL: the map is detached (values no longer written).
 * Synchronises `stream`. */
nebem_status nebem_session_fastvol(nebem_session *s, const nebem_grid *grid, const nebem_axes *axes, double *values,
                                   hipStream_t stream);

/* One step of the dynamic space-charge loop (Sec. 4.3, Algorithm 4; point
 * charges, Sec. 4.2 and Algorithm 2), in place on nq charges:
 *  1. if a re-solve is due (step_index % sc_resolve_every == 0, or with
 *     sc_threshold >= 0 when sum_i |q_i| > sc_threshold): right-hand side b_i = V_i -
 *     phi_q(c_i) on conductor rows, -n_i . E_q(c_i) on dielectric rows
 *     (RHVector with known charges), then sigma = A^-1 b from the resident
 *     factors;
 *  2. E at every charge = panel part (all copies) + k_e sum_{j != i}
 *     q_j (x_i - x_j)/|x_i - x_j|^3 (charges are not copied; coincident
 *     charges are skipped);
 *  3. x_i += sign(q_i) mobility E_i dt (all fields from start-of-step
 *     positions).
 * qx/qy/qz: positions (updated), q: charges (C).  ex/ey/ez (may be NULL):
 * the field used for the move.  Charge-charge sums run in FP32 per pair with
 * FP64 accumulation; the panel part runs in the session's precision. */
nebem_status nebem_spacecharge_step(nebem_session *s, double *qx, double *qy, double *qz, const double *q,
                                    int64_t nq, int32_t step_index, double *ex, double *ey, double *ez,
                                    hipStream_t stream);

/* The same step with the charges reduced to line charges first (Algorithm 3,
 * the cheaper source of Sec. 4.2; voxel grid `vox`, `placement` and line
 * layout as in nebem_voxelize_charges): the lines' potential / normal field
 * at the collocation points replaces the point charges' in step 1, and the
 * charges' own field at every charge is that of nebem_charge_field_lines
 * (far voxels as lines, the 27 voxels around the charge as point charges)
 * in step 2.  Charges outside the grid add no field but still move.
 * *nlines (may be NULL) receives the number of lines.  The session keeps
 * the lines (56 B per occupied voxel), a 32 B-per-charge buffer and the
 * reduction's workspace.  Synchronises `stream`. */
nebem_status nebem_spacecharge_step_lines(nebem_session *s, double *qx, double *qy, double *qz, const double *q,
                                          int64_t nq, int32_t step_index, const nebem_grid *vox, int32_t placement,
                                          double *ex, double *ey, double *ez, int64_t *nlines, hipStream_t stream);

/* ----------------------------------------------------------------- serving
 * Continuous-batching evaluation service over resident sessions.  Clients
 * submit batches of points (host arrays) naming one of the server's
 * sessions; a worker thread admits requests in arrival order while their
 * staging (8 + 4 x nseg doubles per point, nseg = element segments of the
 * geometry, about N x copies / 1.2e5, at most 64) fits the device budget
 * (behind a head of the line that does not fit, up to 64 requests of at
 * most 1/64 of the budget that do fit are admitted past it; with max_large
 * > 0 at most that many large requests are active at once -- first come
 * first served among them -- and a large one beyond it waits at the head
 * like one that does not fit), sorts the
 * points of requests of >= 4096 points into Morton order, cuts the
 * admitted requests into work items of 64 points x one element segment, and
 * evaluates work items of several requests and geometries in each kernel
 * launch (round-robin, up to batch_interactions element-copy x point pairs
 * per launch).  Requests that arrive while others are on the GPU join at the
 * next launch.  A point's result is bit-identical whatever else shares its
 * launches, and bit-identical to nebem_session_eval's (the same element
 * segments, added in the same order). */
typedef struct nebem_server nebem_server;
typedef struct nebem_server_options {
    int64_t hbm_budget;         /* bytes of device staging for admitted requests (2 GiB) */
    double batch_interactions;  /* work per launch, interactions (1e10) */
    int32_t max_items;          /* work items per launch (65536) */
    double large_interactions;  /* a request of at least this much work (interactions) is large (1e11) */
    int32_t max_large;          /* large requests active at once; 0: no limit (1) */
} nebem_server_options;
typedef struct nebem_request_stats {
    double t_submit, t_admit, t_done; /* host steady-clock seconds */
    int64_t points;
} nebem_request_stats;
typedef struct nebem_server_counters {
    int64_t launches, points_done;
    double interactions; /* evaluated so far */
    double busy_s;       /* worker time spent in launches */
    int64_t queued, active;
    int64_t backfilled; /* requests admitted past a head of the line that did not fit */
} nebem_server_counters;

void nebem_server_default_options(nebem_server_options *opt);
/* All sessions must share precision and near_factor and live on the current
 * device; they must outlive the server.  Starts the worker thread. */
nebem_status nebem_server_create(nebem_session *const *sessions, int32_t nsessions, const nebem_server_options *opt,
                                 nebem_server **out);
/* Queues m points (HOST arrays px/py/pz, read until the request completes)
 * on session `geometry`; results go to the HOST arrays phi/ex/ey/ez (any may
 * be NULL).  Returns a ticket.  NEBEM_EBUSY if the request alone exceeds the
 * budget (its staging rounded up, the budget down, to 256 bytes) or the
 * server is shutting down. */
nebem_status nebem_server_submit(nebem_server *s, int32_t geometry, const double *px, const double *py,
                                 const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                                 int64_t *ticket);
/* Blocks until the ticket's request has completed and its results are in the
 * host arrays; fills `stats` (may be NULL).  Each ticket is waited once:
 * NEBEM_EINVAL for an unknown ticket, one already waited for, or one that
 * another thread is waiting for. */
nebem_status nebem_server_wait(nebem_server *s, int64_t ticket, nebem_request_stats *stats);
nebem_status nebem_server_stats(nebem_server *s, nebem_server_counters *out);
/* Finishes every submitted request, stops the worker and frees the server. */
void nebem_server_destroy(nebem_server *s);

/* Thread-local description of the last error (never NULL). */
const char *nebem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NEBEM_H */
