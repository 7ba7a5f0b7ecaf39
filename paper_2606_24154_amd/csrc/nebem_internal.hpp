// nebem_internal.hpp -- declarations shared by the library's translation
// units (host launchers, device record layout, error plumbing).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "nebem.h"

namespace nebem {

constexpr double kEps0 = 8.8541878128e-12;  // vacuum permittivity, F/m
constexpr double kKe = 1.0 / (4.0 * 3.14159265358979323846 * kEps0);

// Derived element record in HBM, 24 doubles (192 B) per element, built once
// per geometry by the prep kernel and streamed through LDS by the field
// kernels.
enum DRec : int {
    R_OX = 0, R_OY, R_OZ,      // corner o
    R_E1X, R_E1Y, R_E1Z,       // unit vector along u
    R_E2X, R_E2Y, R_E2Z,       // unit vector along w
    R_E3X, R_E3Y, R_E3Z,       // unit normal e1 x e2
    R_LX, R_LZ,                // |u|, |w|
    R_HYP, R_IHYP,             // hypotenuse sqrt(lx^2+lz^2) and its inverse
    R_CX, R_CY, R_CZ,          // centroid
    R_DIAM,                    // diameter (rect diagonal / triangle hypotenuse)
    R_AREA,                    // area
    R_KIND,                    // 0 rectangle, 1 right triangle, 2 / 3 right triangle paired with the next one (as double)
    R_JUMP,                    // dielectric diagonal term (eps+ + eps-)/(2 eps0 (eps+ - eps-)), else 0
    R_BC,                      // 0 conductor, 1 dielectric (as double)
    R_STRIDE = 24
};

// Copies of the base cell prepared for kernels: for each of up to 8
// reflection combinations, the reflected lattice vectors M(a1), M(a2), the
// reflected axis mask and the sign carried by sigma.
struct ImgArgs {
    double a1[8][3];
    double a2[8][3];
    double mpos[3];
    double parity[8];
    int axes[8];
    int nref;
    int n1, n2;
    int hole;  // >= 0: the translations with |i1| <= hole and |i2| <= hole are left out (-1: none);
               // honoured by launch_eval only, the other launchers take every copy
};

// thread-local error text
void set_error(const std::string &msg);
nebem_status fail(nebem_status code, const std::string &msg);
nebem_status hip_fail(hipError_t e, const char *what);

#define NEBEM_HIP(call)                                             \
    do {                                                            \
        hipError_t _e = (call);                                     \
        if (_e != hipSuccess) return ::nebem::hip_fail(_e, #call);  \
    } while (0)

nebem_status make_img_args(const nebem_images *im, ImgArgs *out);

// One unit of serving work: up to 64 points of one request against one
// segment of the elements of one resident geometry (device pointers; drec and
// sigma already offset to the segment's first element).
struct WorkItem {
    const double *drec;
    const double *sigma;
    const double *px, *py, *pz;
    double *phi, *ex, *ey, *ez;  // the segment's partial sums (unscaled)
    int n;      // elements in the segment
    int geom;   // index into the image-argument array
    int count;  // points in this item (<= 64)
    int pad;
};

// ---- field kernels (field_kernels.hip)
// Builds derived records; writes bad_count[0] = number of invalid elements,
// bad_count[1] = first invalid index (or n).  bad_count must be zeroed/set
// to {0, n} by the caller.
void launch_prep(const nebem_panels *p, double *drec, int *bad, hipStream_t s);
// FastVolume grid (fastvol_kernels.hip): nodes origin + (i, j, k) * step,
// n[0] x n[1] x n[2] of them, node values interleaved 4 per node.
struct GridArgs {
    double origin[3], step[3], inv_step[3];
    int n[3];
};
void launch_grid_nodes(const GridArgs &g, double *px, double *py, double *pz, hipStream_t s);
// Graded FastVolume grid: node (i, j, k) at (ax[0][i], ax[1][j], ax[2][k]),
// each axis strictly increasing (device arrays), same node order and value
// interleaving as the regular grid.
struct AxesArgs {
    const double *ax[3];
    int n[3];
};
void launch_axes_nodes(const AxesArgs &g, double *px, double *py, double *pz, hipStream_t s);
void launch_axes_check(const AxesArgs &g, int *bad, hipStream_t s);  // bad[0] = 1 on a bad axis
void launch_fastvol_interp_axes(const AxesArgs &g, const double *values, const double *px, const double *py,
                                const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                                hipStream_t s);
void launch_interleave4(const double *s0, const double *s1, const double *s2, const double *s3, int64_t nn,
                        double *values, hipStream_t s);
void launch_fastvol_interp(const GridArgs &g, const double *values, const double *px, const double *py,
                           const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                           hipStream_t s);

// Point charges -> line charges (line_kernels.hip).  Workspace layout of
// one reduction (byte offsets); after voxel_lines it holds the charges
// sorted by voxel (kout keys, iout charge indices), the runs' starts, the
// count of charges inside the grid (nvalid, device int) and, at `flag`, the
// lines' voxel keys.
struct VoxelLayout {
    size_t kin, kout, iin, iout, flag, pos, start, nvalid, sortw, sort_bytes, scanw, scan_bytes, total;
};
bool voxel_layout(int nq, VoxelLayout &L);
size_t voxel_workspace(int nq);  // 0 on error
// lines (7 doubles each) written only when *nlines <= max_lines; weighted:
// lines at the |q|-weighted mean x, y of their charges, else through the
// voxel centre; synchronises the stream.
hipError_t voxel_lines(const double *qx, const double *qy, const double *qz, const double *q, int nq,
                       const GridArgs &g, int weighted, double *lines, int64_t max_lines, int64_t *nlines,
                       int64_t *outside, void *ws, size_t ws_bytes, hipStream_t s);
// Field of the charges at themselves from their lines (ws as left by
// voxel_lines with these charges and lines): the lines of every voxel except
// the charge's own and the 26 around it, plus those voxels' charges one by
// one; written to ex/ey/ez.
void launch_line_field_at_charges(const double *lines, int64_t nl, const void *ws, const GridArgs &g,
                                  const double *qx, const double *qy, const double *qz, const double *q, int nq,
                                  double *ex, double *ey, double *ez, hipStream_t s);
void launch_line_field(const double *lines, int64_t nl, const double *px, const double *py, const double *pz,
                       int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t s);
// Right-hand side with line charges at the collocation points: b = b0 - phi
// (conductor rows) or b0 - n . E (interface rows); work: 7 n doubles
void launch_line_rhs(const double *drec, int64_t n, const double *lines, int64_t nl, const double *b0, double *work,
                     double *b, hipStream_t s);

// o_c[i] += add[c m + i] for each non-null o_c
void launch_add4(const double *add, int64_t m, double *o0, double *o1, double *o2, double *o3, hipStream_t s);
// sbar[p] = sum_{map[j] == p} sigma_j A_j / A_p (records drec, prec), in
// element order; *bad (device int, cleared by the caller) set if a map entry
// is outside [0, np); ws of prim_density_workspace(n) bytes (0 on error)
size_t prim_density_workspace(int64_t n);
hipError_t launch_prim_density(const double *drec, const double *sigma, const int32_t *map, int64_t n,
                               const double *prec, int64_t np, double *sbar, int *bad, void *ws, size_t ws_bytes,
                               hipStream_t s);

// Output columns of a several-column evaluation: component c (phi, ex, ey,
// ez) of column k at c[c] + k * stride; a null c[c] is not stored.
struct OutCols {
    double *c[4];
    int64_t stride;
};
constexpr int kMultiCols = 4;  // density columns per evaluation launch

// Element segments of an evaluation (field_kernels.hip): nseg contiguous
// ranges of segsz elements (the last may be shorter), about kSegWork
// interactions per point each; a function of the element count and copies
// only, shared by every evaluation path and the server.
constexpr double kSegWork = 1.2e5;
constexpr int kMaxSeg = 64;
struct SegPlan {
    int nseg, segsz;
};
int64_t img_copies(const ImgArgs &img);  // copies per element (reflections x translations, minus any hole)
SegPlan seg_plan(int64_t n, const ImgArgs &img);
// In the evaluation launchers, mixed != 0: copies beyond the far-field tiers
// (rectangles >= 24 D, triangles >= 48 D, never below near_factor D) use the
// FP64 monopole + FP32 correction far field, nearer ones the exact FP64
// closed forms; mixed == 0: the exact FP64 closed forms everywhere.
// One launch over all segments: segment y's sums (times `scale`) go to the
// outputs + y * seg_stride (nseg == 1, scale k_e: the final results).
void launch_eval_seg(const double *drec, const double *sigma, int64_t n, const SegPlan &sp, const ImgArgs &img,
                     int mixed, double near_factor, const double *px, const double *py, const double *pz, int64_t m,
                     double scale, double *phi, double *ex, double *ey, double *ez, int64_t seg_stride, hipStream_t s);
// ncol <= kMultiCols columns of sigma (column k at sigma + k sig_stride)
void launch_eval_multi_seg(const double *drec, const double *sigma, int64_t n, int64_t sig_stride, int ncol,
                           const SegPlan &sp, const ImgArgs &img, int mixed, double near_factor, const double *px,
                           const double *py, const double *pz, int64_t m, double scale, const OutCols &out,
                           int64_t seg_stride, hipStream_t s);
// out.c[c][k stride + i] = k_e * (0 + sum_s part[s seg_stride + (4k + c) m + i]), in segment order
void launch_reduce_segments(const double *part, int nseg, int ncol, int64_t m, int64_t seg_stride,
                            const OutCols &out, hipStream_t s);

// ---- Morton order of points (order_kernels.hip)
bool eval_ordering_pays(int64_t m);
// Morton order of m points: s{x,y,z}[k] = p{x,y,z}[perm[k]]; ws of
// order_points_workspace(m) bytes (0 on error)
size_t order_points_workspace(int64_t m);
hipError_t launch_order_points(const double *px, const double *py, const double *pz, int64_t m, double *sx,
                               double *sy, double *sz, int *perm, void *ws, size_t ws_bytes, hipStream_t s);
// d_j[perm[k]] = src[j * m + k] for each non-null d_j (j = 0..3)
void launch_unorder4(const double *src, const int *perm, int64_t m, double *d0, double *d1, double *d2, double *d3,
                     hipStream_t s);

// ---- the evaluation driver (order_kernels.hip), used by every evaluation
// entry point: ncol density columns (column k at sigma + k n), outputs m x
// ncol column-major per component (null: not stored).  Points are taken in
// chunks whose workspace fits ws_bytes; chunks of >= 4096 points are
// evaluated in Morton order; every element segment of a chunk is one grid
// row, and the segments' partial sums are reduced in segment order.  No
// result bit depends on the chunking, the ordering or the other points.
// eval_workspace: the workspace that lets the driver take its preferred
// chunk (0 when none is needed).
size_t eval_workspace(int64_t n, const ImgArgs &img, int64_t m, int ncol);
// smallest workspace with which run_eval accepts the call
size_t eval_workspace_min(int64_t n, const ImgArgs &img, int64_t m, int ncol);
hipError_t run_eval(const double *drec, const double *sigma, int64_t n, int ncol, const ImgArgs &img, int mixed,
                    double near_factor, const double *px, const double *py, const double *pz, int64_t m, double *phi,
                    double *ex, double *ey, double *ez, void *ws, size_t ws_bytes, hipStream_t s);
// work items (one wave each) the device holds at once: CUs x resident
// workgroups of the items kernel per CU (1 when the query fails)
int eval_items_slots(int mixed);
// items/imgs in device memory; one 64-lane workgroup per item
void launch_eval_items(const WorkItem *items, int nitems, const ImgArgs *imgs, int mixed, double near_factor,
                       hipStream_t s);
// A (n x n col-major), exact closed forms.  cx/cy/cz may be null (centroids).
void launch_assemble(const double *drec, int64_t n, const ImgArgs &img, const double *cx, const double *cy,
                     const double *cz, double *A, hipStream_t s);

}  // namespace nebem
