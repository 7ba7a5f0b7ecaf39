// api.hip -- the C-ABI of libnebem (see include/nebem.h): argument checks,
// stream-ordered temporaries, geometry preparation and the solve drivers.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_util.hpp"
#include "lu_internal.hpp"
#include "nebem_internal.hpp"

namespace nebem {

static thread_local std::string g_err = "no error";

void set_error(const std::string &msg) { g_err = msg; }
nebem_status fail(nebem_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}
nebem_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NEBEM_ENOMEM : NEBEM_EDEVICE;
}

nebem_status make_img_args(const nebem_images *im, ImgArgs *o)
{
    std::memset(o, 0, sizeof(*o));
    o->hole = -1;
    if (!im) {
        o->nref = 1;
        o->parity[0] = 1.0;
        return NEBEM_OK;
    }
    if (im->n1 < 0 || im->n2 < 0 || im->n1 > 64 || im->n2 > 64)
        return fail(NEBEM_EINVAL, "images: n1, n2 must be in [0, 64]");
    if (im->mirror_mask < 0 || im->mirror_mask > 7) return fail(NEBEM_EINVAL, "images: mirror_mask must be in [0, 7]");
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(im->a1[k]) || !std::isfinite(im->a2[k]) || !std::isfinite(im->mirror_pos[k]))
            return fail(NEBEM_EINVAL, "images: non-finite lattice vector or mirror position");
        if ((im->mirror_mask >> k & 1) && im->mirror_parity[k] != 1 && im->mirror_parity[k] != -1)
            return fail(NEBEM_EINVAL, "images: mirror_parity must be +1 or -1");
    }
    int active[3], na = 0;
    for (int k = 0; k < 3; ++k)
        if (im->mirror_mask >> k & 1) active[na++] = k;
    o->nref = 1 << na;
    o->n1 = im->n1;
    o->n2 = im->n2;
    for (int k = 0; k < 3; ++k) o->mpos[k] = im->mirror_pos[k];
    for (int r = 0; r < o->nref; ++r) {
        int axes = 0;
        double par = 1.0;
        for (int b = 0; b < na; ++b)
            if (r >> b & 1) {
                axes |= 1 << active[b];
                par *= (double)im->mirror_parity[active[b]];
            }
        o->axes[r] = axes;
        o->parity[r] = par;
        for (int k = 0; k < 3; ++k) {
            const double f = (axes >> k & 1) ? -1.0 : 1.0;
            o->a1[r][k] = f * im->a1[k];
            o->a2[r][k] = f * im->a2[k];
        }
    }
    return NEBEM_OK;
}

nebem_status check_panels(const nebem_panels *p)
{
    if (!p) return fail(NEBEM_EINVAL, "panels is NULL");
    if (p->n < 0 || p->n > (int64_t)INT_MAX / 2) return fail(NEBEM_EINVAL, "panels: n out of range");
    if (p->n == 0) return NEBEM_OK;
    if (!p->kind || !p->ox || !p->oy || !p->oz || !p->ux || !p->uy || !p->uz || !p->wx || !p->wy || !p->wz ||
        !p->bc || !p->eps_pos || !p->eps_neg)
        return fail(NEBEM_EINVAL, "panels: NULL array");
    return NEBEM_OK;
}

static const nebem_options &opts_or_default(const nebem_options *opt, nebem_options &tmp)
{
    if (opt) return *opt;
    nebem_default_options(&tmp);
    return tmp;
}

nebem_status check_options(const nebem_options &o)
{
    if (o.precision != NEBEM_FP64 && o.precision != NEBEM_MIXED) return fail(NEBEM_EINVAL, "options: bad precision");
    if (!(o.near_factor >= 1.0) || !std::isfinite(o.near_factor))
        return fail(NEBEM_EINVAL, "options: near_factor must be >= 1");
    if (!(o.ir_tol > 0.0) || o.ir_max_iter < 0) return fail(NEBEM_EINVAL, "options: bad refinement settings");
    return NEBEM_OK;
}

// Derived element records for `p` in a stream-ordered buffer; validates the
// elements (synchronises the stream to read the verdict).
nebem_status derive(const nebem_panels *p, hipStream_t s, DevBuf &drec)
{
    NEBEM_HIP(drec.alloc((size_t)p->n * R_STRIDE * sizeof(double), s));
    DevBuf bad;
    NEBEM_HIP(bad.alloc(2 * sizeof(int), s));
    NEBEM_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    NEBEM_HIP(hipMemsetAsync(bad.as<int>() + 1, 0x7f, sizeof(int), s));
    launch_prep(p, drec.as<double>(), bad.as<int>(), s);
    NEBEM_HIP(hipGetLastError());
    int h[2] = {0, 0};
    NEBEM_HIP(hipMemcpyAsync(h, bad.p, sizeof(h), hipMemcpyDeviceToHost, s));
    NEBEM_HIP(hipStreamSynchronize(s));
    if (h[0] != 0) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "%d invalid panel(s), first at index %d (kind/bc out of range, zero or non-perpendicular "
                      "edges, non-finite data, or bad dielectric permittivities)",
                      h[0], h[1]);
        return fail(NEBEM_EINVAL, buf);
    }
    return NEBEM_OK;
}

// host permutation from LAPACK-style sequential row swaps
void pivots_to_perm(const std::vector<int> &ipiv, std::vector<int> &perm)
{
    const int n = (int)ipiv.size();
    perm.resize(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int k = 0; k < n; ++k) std::swap(perm[k], perm[ipiv[k]]);
}

nebem_status voxel_grid_args(const nebem_grid *vox, GridArgs &g)
{
    if (!vox) return fail(NEBEM_EINVAL, "voxelize: NULL grid");
    for (int a = 0; a < 3; ++a) {
        if (vox->n[a] < 1) return fail(NEBEM_EINVAL, "voxelize: fewer than 1 voxel on an axis");
        if (!(vox->step[a] > 0.0) || !std::isfinite(vox->step[a]) || !std::isfinite(vox->origin[a]))
            return fail(NEBEM_EINVAL, "voxelize: step must be finite and > 0, origin finite");
        g.origin[a] = vox->origin[a];
        g.step[a] = vox->step[a];
        g.inv_step[a] = 1.0 / vox->step[a];
        g.n[a] = vox->n[a];
    }
    const int64_t nn = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (nn >= (int64_t)0xffffffffLL) return fail(NEBEM_EINVAL, "voxelize: too many voxels (>= 2^32 - 1)");
    return NEBEM_OK;
}

// one evaluation through the driver, with a stream-ordered workspace of
// the driver's preferred size; outputs overwritten
nebem_status eval_with_workspace(const double *drec, const double *sigma, int64_t n, int ncol, const ImgArgs &ia,
                                 int mixed, double near_factor, const double *px, const double *py, const double *pz,
                                 int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t stream,
                                 const char *what)
{
    const size_t wb = eval_workspace(n, ia, m, ncol);
    DevBuf ws;
    if (wb && ws.alloc(wb, stream) != hipSuccess)
        return fail(NEBEM_ENOMEM, std::string(what) + ": evaluation workspace");
    NEBEM_HIP(run_eval(drec, sigma, n, ncol, ia, mixed, near_factor, px, py, pz, m, phi, ex, ey, ez, ws.p, wb,
                       stream));
    return NEBEM_OK;
}

}  // namespace nebem

using namespace nebem;

extern "C" {

void nebem_default_options(nebem_options *o)
{
    if (!o) return;
    o->precision = NEBEM_FP64;
    o->near_factor = 4.0;
    o->ir_tol = 1e-10;
    o->ir_max_iter = 30;
    o->sc_dt = 1e-12;
    o->sc_mobility = 1e-4;
    o->sc_resolve_every = 10;
    o->sc_threshold = -1.0;
}

const char *nebem_last_error(void) { return g_err.c_str(); }

nebem_status nebem_eval(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                        const double *px, const double *py, const double *pz, int64_t m, double *phi, double *ex,
                        double *ey, double *ez, const nebem_options *opt, hipStream_t stream)
{
    nebem_status st = check_panels(panels);
    if (st) return st;
    nebem_options tmp;
    const nebem_options &o = opts_or_default(opt, tmp);
    if ((st = check_options(o))) return st;
    if (m < 0 || m > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "eval: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!px || !py || !pz) return fail(NEBEM_EINVAL, "eval: NULL point array");
    if (panels->n > 0 && !sigma) return fail(NEBEM_EINVAL, "eval: NULL sigma");
    ImgArgs ia;
    if ((st = make_img_args(images, &ia))) return st;
    DevBuf drec;
    if ((st = derive(panels, stream, drec))) return st;
    return eval_with_workspace(drec.as<double>(), sigma, panels->n, 1, ia, o.precision == NEBEM_MIXED,
                               o.near_factor, px, py, pz, m, phi, ex, ey, ez, stream, "eval");
}

nebem_status nebem_eval_multi(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                              int64_t nsig, const double *px, const double *py, const double *pz, int64_t m,
                              double *phi, double *ex, double *ey, double *ez, const nebem_options *opt,
                              hipStream_t stream)
{
    nebem_status st = check_panels(panels);
    if (st) return st;
    nebem_options tmp;
    const nebem_options &o = opts_or_default(opt, tmp);
    if ((st = check_options(o))) return st;
    if (m < 0 || m > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "eval_multi: m out of range");
    if (nsig < 0 || nsig > 64) return fail(NEBEM_EINVAL, "eval_multi: nsig out of range (0..64)");
    if (m == 0 || nsig == 0) return NEBEM_OK;
    if (!px || !py || !pz) return fail(NEBEM_EINVAL, "eval_multi: NULL point array");
    if (panels->n > 0 && !sigma) return fail(NEBEM_EINVAL, "eval_multi: NULL sigma");
    if ((uint64_t)m * (uint64_t)nsig > (uint64_t)1 << 40) return fail(NEBEM_EINVAL, "eval_multi: m * nsig too large");
    ImgArgs ia;
    if ((st = make_img_args(images, &ia))) return st;
    DevBuf drec;
    if ((st = derive(panels, stream, drec))) return st;
    return eval_with_workspace(drec.as<double>(), sigma, panels->n, (int)nsig, ia, o.precision == NEBEM_MIXED,
                               o.near_factor, px, py, pz, m, phi, ex, ey, ez, stream, "eval_multi");
}

nebem_status nebem_eval_adaptive(const nebem_panels *panels, const nebem_panels *prims, const int32_t *elem_prim,
                                 int32_t prim_after, const nebem_images *images, const double *sigma, const double *px,
                                 const double *py, const double *pz, int64_t m, double *phi, double *ex, double *ey,
                                 double *ez, const nebem_options *opt, hipStream_t stream)
{
    if (prim_after < 0)
        return nebem_eval(panels, images, sigma, px, py, pz, m, phi, ex, ey, ez, opt, stream);
    nebem_status st = check_panels(panels);
    if (st) return st;
    if ((st = check_panels(prims))) return st;
    nebem_options tmp;
    const nebem_options &o = opts_or_default(opt, tmp);
    if ((st = check_options(o))) return st;
    if (m < 0 || m > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "eval_adaptive: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!px || !py || !pz) return fail(NEBEM_EINVAL, "eval_adaptive: NULL point array");
    const int64_t n = panels->n, np = prims->n;
    if (n > 0 && (!sigma || !elem_prim)) return fail(NEBEM_EINVAL, "eval_adaptive: NULL sigma or elem_prim");
    ImgArgs ia;
    if ((st = make_img_args(images, &ia))) return st;
    const int mixed = o.precision == NEBEM_MIXED;
    // near copies: every element, lattice |i1|, |i2| <= prim_after
    ImgArgs near = ia;
    near.n1 = ia.n1 < prim_after ? ia.n1 : prim_after;
    near.n2 = ia.n2 < prim_after ? ia.n2 : prim_after;
    DevBuf drec;
    if ((st = derive(panels, stream, drec))) return st;
    if (n == 0) {
        // no elements: nothing near; the far pass below has no charge either
        for (double *out : {phi, ex, ey, ez})
            if (out) NEBEM_HIP(hipMemsetAsync(out, 0, (size_t)m * sizeof(double), stream));
        return NEBEM_OK;
    }
    if ((st = eval_with_workspace(drec.as<double>(), sigma, n, 1, near, mixed, o.near_factor, px, py, pz, m, phi, ex,
                                  ey, ez, stream, "eval_adaptive")))
        return st;
    if (prim_after >= ia.n1 && prim_after >= ia.n2) return NEBEM_OK;  // no far copies
    if (np == 0) return fail(NEBEM_EINVAL, "eval_adaptive: no primitives");
    // primitive-averaged densities: sigma_p = sum_{j in p} sigma_j A_j / A_p
    DevBuf prec, dsbar, dbad, far, pws;
    if ((st = derive(prims, stream, prec))) return st;
    NEBEM_HIP(dsbar.alloc((size_t)np * sizeof(double), stream));
    NEBEM_HIP(dbad.alloc(sizeof(int), stream));
    NEBEM_HIP(hipMemsetAsync(dbad.p, 0, sizeof(int), stream));
    const size_t pwb = prim_density_workspace(n);
    if (!pwb || pws.alloc(pwb, stream) != hipSuccess) return fail(NEBEM_ENOMEM, "eval_adaptive: workspace");
    NEBEM_HIP(launch_prim_density(drec.as<double>(), sigma, elem_prim, n, prec.as<double>(), np, dsbar.as<double>(),
                                  static_cast<int *>(dbad.p), pws.p, pwb, stream));
    int hbad = 0;
    NEBEM_HIP(hipMemcpyAsync(&hbad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    NEBEM_HIP(hipStreamSynchronize(stream));
    if (hbad) return fail(NEBEM_EINVAL, "eval_adaptive: elem_prim out of range");
    NEBEM_HIP(far.alloc((size_t)4 * m * sizeof(double), stream));
    ImgArgs farimg = ia;
    farimg.hole = prim_after;
    double *f = far.as<double>();
    const size_t mm = (size_t)m;
    if ((st = eval_with_workspace(prec.as<double>(), dsbar.as<double>(), np, 1, farimg, mixed, o.near_factor, px, py,
                                  pz, m, phi ? f : nullptr, ex ? f + mm : nullptr, ey ? f + 2 * mm : nullptr,
                                  ez ? f + 3 * mm : nullptr, stream, "eval_adaptive")))
        return st;
    launch_add4(f, m, phi, ex, ey, ez, stream);
    NEBEM_HIP(hipGetLastError());
    NEBEM_HIP(hipStreamSynchronize(stream));  // the scratch buffers are freed on return
    return NEBEM_OK;
}

static nebem_status grid_args(const nebem_grid *grid, GridArgs &g, int64_t &nn)
{
    if (!grid) return fail(NEBEM_EINVAL, "fastvol: NULL grid");
    nn = 1;
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 2) return fail(NEBEM_EINVAL, "fastvol: fewer than 2 nodes on an axis");
        if (!(grid->step[a] > 0.0) || !std::isfinite(grid->step[a]) || !std::isfinite(grid->origin[a]))
            return fail(NEBEM_EINVAL, "fastvol: step must be finite and > 0, origin finite");
        nn *= grid->n[a];
        if (nn > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "fastvol: too many nodes");
        g.origin[a] = grid->origin[a];
        g.step[a] = grid->step[a];
        g.inv_step[a] = 1.0 / grid->step[a];
        g.n[a] = grid->n[a];
    }
    return NEBEM_OK;
}

nebem_status nebem_fastvol_build(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                                 const nebem_grid *grid, double *values, const nebem_options *opt,
                                 hipStream_t stream)
{
    GridArgs g;
    int64_t nn = 0;
    nebem_status st = grid_args(grid, g, nn);
    if (st) return st;
    if (!values) return fail(NEBEM_EINVAL, "fastvol_build: NULL values");
    if ((uintptr_t)values % 16) return fail(NEBEM_EINVAL, "fastvol_build: values must be 16-byte aligned");
    DevBuf tmp;
    if (tmp.alloc((size_t)nn * 7 * sizeof(double), stream) != hipSuccess)
        return fail(NEBEM_ENOMEM, "fastvol_build: node buffers");
    double *t = tmp.as<double>();
    const size_t q = (size_t)nn;
    launch_grid_nodes(g, t, t + q, t + 2 * q, stream);
    NEBEM_HIP(hipGetLastError());
    if ((st = nebem_eval(panels, images, sigma, t, t + q, t + 2 * q, nn, t + 3 * q, t + 4 * q, t + 5 * q, t + 6 * q,
                         opt, stream)))
        return st;
    launch_interleave4(t + 3 * q, t + 4 * q, t + 5 * q, t + 6 * q, nn, values, stream);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

nebem_status nebem_fastvol_interp(const nebem_grid *grid, const double *values, const double *px, const double *py,
                                  const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                                  hipStream_t stream)
{
    GridArgs g;
    int64_t nn = 0;
    nebem_status st = grid_args(grid, g, nn);
    if (st) return st;
    if (m < 0 || m > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "fastvol_interp: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!values || !px || !py || !pz) return fail(NEBEM_EINVAL, "fastvol_interp: NULL argument");
    if ((uintptr_t)values % 16) return fail(NEBEM_EINVAL, "fastvol_interp: values must be 16-byte aligned");
    launch_fastvol_interp(g, values, px, py, pz, m, phi, ex, ey, ez, stream);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

static nebem_status axes_args(const nebem_axes *grid, AxesArgs &g, int64_t &nn)
{
    if (!grid) return fail(NEBEM_EINVAL, "fastvol_axes: NULL grid");
    if (!grid->x || !grid->y || !grid->z) return fail(NEBEM_EINVAL, "fastvol_axes: NULL axis");
    g.ax[0] = grid->x;
    g.ax[1] = grid->y;
    g.ax[2] = grid->z;
    nn = 1;
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 2) return fail(NEBEM_EINVAL, "fastvol_axes: fewer than 2 nodes on an axis");
        g.n[a] = grid->n[a];
        nn *= grid->n[a];
        if (nn > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "fastvol_axes: too many nodes");
    }
    return NEBEM_OK;
}

nebem_status nebem_fastvol_build_axes(const nebem_panels *panels, const nebem_images *images, const double *sigma,
                                      const nebem_axes *grid, double *values, const nebem_options *opt,
                                      hipStream_t stream)
{
    AxesArgs g;
    int64_t nn = 0;
    nebem_status st = axes_args(grid, g, nn);
    if (st) return st;
    if (!values) return fail(NEBEM_EINVAL, "fastvol_build_axes: NULL values");
    if ((uintptr_t)values % 16) return fail(NEBEM_EINVAL, "fastvol_build_axes: values must be 16-byte aligned");
    DevBuf tmp, dbad;
    if (tmp.alloc((size_t)nn * 7 * sizeof(double), stream) != hipSuccess ||
        dbad.alloc(sizeof(int), stream) != hipSuccess)
        return fail(NEBEM_ENOMEM, "fastvol_build_axes: node buffers");
    NEBEM_HIP(hipMemsetAsync(dbad.p, 0, sizeof(int), stream));
    launch_axes_check(g, static_cast<int *>(dbad.p), stream);
    NEBEM_HIP(hipGetLastError());
    int hbad = 0;
    NEBEM_HIP(hipMemcpyAsync(&hbad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    NEBEM_HIP(hipStreamSynchronize(stream));
    if (hbad) return fail(NEBEM_EINVAL, "fastvol_build_axes: an axis is not strictly increasing and finite");
    double *t = tmp.as<double>();
    const size_t q = (size_t)nn;
    launch_axes_nodes(g, t, t + q, t + 2 * q, stream);
    NEBEM_HIP(hipGetLastError());
    if ((st = nebem_eval(panels, images, sigma, t, t + q, t + 2 * q, nn, t + 3 * q, t + 4 * q, t + 5 * q, t + 6 * q,
                         opt, stream)))
        return st;
    launch_interleave4(t + 3 * q, t + 4 * q, t + 5 * q, t + 6 * q, nn, values, stream);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

nebem_status nebem_fastvol_interp_axes(const nebem_axes *grid, const double *values, const double *px,
                                       const double *py, const double *pz, int64_t m, double *phi, double *ex,
                                       double *ey, double *ez, hipStream_t stream)
{
    AxesArgs g;
    int64_t nn = 0;
    nebem_status st = axes_args(grid, g, nn);
    if (st) return st;
    if (m < 0 || m > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "fastvol_interp_axes: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!values || !px || !py || !pz) return fail(NEBEM_EINVAL, "fastvol_interp_axes: NULL argument");
    if ((uintptr_t)values % 16) return fail(NEBEM_EINVAL, "fastvol_interp_axes: values must be 16-byte aligned");
    launch_fastvol_interp_axes(g, values, px, py, pz, m, phi, ex, ey, ez, stream);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

nebem_status nebem_voxelize_charges(const double *qx, const double *qy, const double *qz, const double *q,
                                    int64_t nq, const nebem_grid *vox, int32_t placement, double *lines,
                                    int64_t max_lines, int64_t *nlines, int64_t *outside, hipStream_t stream)
{
    GridArgs g;
    if (!nlines) return fail(NEBEM_EINVAL, "voxelize: NULL nlines");
    *nlines = 0;
    if (outside) *outside = 0;
    nebem_status st = voxel_grid_args(vox, g);
    if (st) return st;
    if (placement != NEBEM_LINE_CENTRE && placement != NEBEM_LINE_WEIGHTED)
        return fail(NEBEM_EINVAL, "voxelize: unknown line placement");
    if (nq < 0 || nq > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "voxelize: nq out of range");
    if (max_lines < 0) return fail(NEBEM_EINVAL, "voxelize: negative max_lines");
    if (nq == 0) return NEBEM_OK;
    if (!qx || !qy || !qz || !q) return fail(NEBEM_EINVAL, "voxelize: NULL charge array");
    const size_t wb = voxel_workspace((int)nq);
    DevBuf ws;
    if (!wb || ws.alloc(wb, stream) != hipSuccess) return fail(NEBEM_ENOMEM, "voxelize: workspace");
    NEBEM_HIP(voxel_lines(qx, qy, qz, q, (int)nq, g, placement == NEBEM_LINE_WEIGHTED, lines, max_lines, nlines,
                          outside, ws.p, wb, stream));
    if (*nlines > max_lines) return fail(NEBEM_EINVAL, "voxelize: more occupied voxels than max_lines (*nlines)");
    return NEBEM_OK;
}

nebem_status nebem_charge_field_lines(const double *qx, const double *qy, const double *qz, const double *q,
                                      int64_t nq, const nebem_grid *vox, int32_t placement, double *ex, double *ey,
                                      double *ez, int64_t *nlines, hipStream_t stream)
{
    if (nlines) *nlines = 0;
    GridArgs g;
    nebem_status st = voxel_grid_args(vox, g);
    if (st) return st;
    if (placement != NEBEM_LINE_CENTRE && placement != NEBEM_LINE_WEIGHTED)
        return fail(NEBEM_EINVAL, "charge_field_lines: unknown line placement");
    if (nq < 0 || nq > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "charge_field_lines: nq out of range");
    if (nq == 0) return NEBEM_OK;
    if (!qx || !qy || !qz || !q || !ex || !ey || !ez)
        return fail(NEBEM_EINVAL, "charge_field_lines: NULL argument");
    const int64_t nvox = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t cap = nq < nvox ? nq : nvox;
    const size_t wb = voxel_workspace((int)nq);
    DevBuf ws, lines;
    if (!wb || ws.alloc(wb, stream) != hipSuccess ||
        lines.alloc((size_t)cap * 7 * sizeof(double), stream) != hipSuccess)
        return fail(NEBEM_ENOMEM, "charge_field_lines: workspace");
    int64_t nl = 0;
    NEBEM_HIP(voxel_lines(qx, qy, qz, q, (int)nq, g, placement == NEBEM_LINE_WEIGHTED, lines.as<double>(), cap, &nl,
                          nullptr, ws.p, wb, stream));
    launch_line_field_at_charges(lines.as<double>(), nl, ws.p, g, qx, qy, qz, q, (int)nq, ex, ey, ez, stream);
    NEBEM_HIP(hipGetLastError());
    if (nlines) *nlines = nl;
    return NEBEM_OK;
}

nebem_status nebem_line_field(const double *lines, int64_t nlines, const double *px, const double *py,
                              const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                              hipStream_t stream)
{
    if (nlines < 0 || nlines > (int64_t)INT_MAX) return fail(NEBEM_EINVAL, "line_field: nlines out of range");
    if (m < 0 || m > (int64_t)INT_MAX - 256) return fail(NEBEM_EINVAL, "line_field: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!px || !py || !pz || (nlines > 0 && !lines)) return fail(NEBEM_EINVAL, "line_field: NULL argument");
    launch_line_field(lines, nlines, px, py, pz, m, phi, ex, ey, ez, stream);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

nebem_status nebem_assemble(const nebem_panels *panels, const nebem_images *images, const double *cx,
                            const double *cy, const double *cz, const nebem_options *opt, double *A,
                            hipStream_t stream)
{
    nebem_status st = check_panels(panels);
    if (st) return st;
    nebem_options tmp;
    const nebem_options &o = opts_or_default(opt, tmp);
    if ((st = check_options(o))) return st;
    if (!A) return fail(NEBEM_EINVAL, "assemble: NULL matrix");
    if ((cx == nullptr) != (cy == nullptr) || (cx == nullptr) != (cz == nullptr))
        return fail(NEBEM_EINVAL, "assemble: collocation arrays must be all NULL or all set");
    if (panels->n == 0) return NEBEM_OK;
    ImgArgs ia;
    if ((st = make_img_args(images, &ia))) return st;
    DevBuf drec;
    if ((st = derive(panels, stream, drec))) return st;
    launch_assemble(drec.as<double>(), panels->n, ia, cx, cy, cz, A, stream);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

nebem_status nebem_solve(double *A, int64_t n, const double *b, int64_t nrhs, double *sigma, int32_t *ipiv,
                         const nebem_options *opt, nebem_solve_info *info, hipStream_t stream)
{
    nebem_options tmp;
    const nebem_options &o = opts_or_default(opt, tmp);
    nebem_status st;
    if ((st = check_options(o))) return st;
    if (n < 0 || n > 65536 * 4) return fail(NEBEM_EINVAL, "solve: n out of range");
    if (nrhs < 0 || nrhs > 4096) return fail(NEBEM_EINVAL, "solve: nrhs out of range");
    if (info) {
        info->ir_iters = 0;
        info->rel_resid = -1.0;
    }
    if (n == 0 || nrhs == 0) return NEBEM_OK;
    if (!A || !b || !sigma || !ipiv) return fail(NEBEM_EINVAL, "solve: NULL argument");
    const int nn = (int)n;
    std::vector<int> perm;
    DevBuf dperm;
    NEBEM_HIP(dperm.alloc((size_t)nn * sizeof(int), stream));
    if (o.precision == NEBEM_FP64) {
        // The LU solution is refined in FP64 against a copy of the unfactored
        // matrix (the factorisation overwrites A); without room for the copy
        // the LU solution is returned as it is.
        DevBuf acopy, bcopy64;
        bool refine = acopy.alloc((size_t)nn * nn * sizeof(double), stream) == hipSuccess;
        if (!refine) {
            (void)hipGetLastError();
            acopy.p = nullptr;
        }
        const double *bb = b;
        if (refine) {
            NEBEM_HIP(hipMemcpyAsync(acopy.p, A, (size_t)nn * nn * sizeof(double), hipMemcpyDeviceToDevice, stream));
            if (sigma == b) {  // refinement reads b after x is written
                NEBEM_HIP(bcopy64.alloc((size_t)nn * nrhs * sizeof(double), stream));
                NEBEM_HIP(hipMemcpyAsync(bcopy64.p, b, (size_t)nn * nrhs * sizeof(double), hipMemcpyDeviceToDevice,
                                         stream));
                bb = bcopy64.as<double>();
            }
        }
        if ((st = factor_fp64(A, nn, ipiv, perm, stream))) return st;
        NEBEM_HIP(hipMemcpyAsync(dperm.p, perm.data(), (size_t)nn * sizeof(int), hipMemcpyHostToDevice, stream));
        if ((st = solve_fp64(A, nn, dperm.as<int>(), b, (int)nrhs, sigma, stream))) return st;
        if (refine) {
            nebem_solve_info agg = {0, 0.0};
            for (int64_t q = 0; q < nrhs; ++q) {
                nebem_solve_info ci;
                if ((st = refine_fp64(acopy.as<double>(), A, dperm.as<int>(), nn, bb + q * n, sigma + q * n,
                                      kFp64RefineSteps, &ci, stream)))
                    return st;
                agg.ir_iters = ci.ir_iters > agg.ir_iters ? ci.ir_iters : agg.ir_iters;
                agg.rel_resid = ci.rel_resid > agg.rel_resid ? ci.rel_resid : agg.rel_resid;
            }
            if (info) *info = agg;
        }
        NEBEM_HIP(hipStreamSynchronize(stream));  // perm (host) must outlive the copy
        return NEBEM_OK;
    }
    DevBuf a32, scale, bcopy;
    NEBEM_HIP(a32.alloc((size_t)nn * nn * sizeof(float), stream));
    NEBEM_HIP(scale.alloc((size_t)nn * sizeof(double), stream));
    if ((st = factor_mixed(A, nn, a32.as<float>(), scale.as<double>(), ipiv, perm, stream))) return st;
    NEBEM_HIP(hipMemcpyAsync(dperm.p, perm.data(), (size_t)nn * sizeof(int), hipMemcpyHostToDevice, stream));
    const double *bb = b;
    if (sigma == b) {  // the refinement reads b after writing x
        NEBEM_HIP(bcopy.alloc((size_t)nn * nrhs * sizeof(double), stream));
        NEBEM_HIP(hipMemcpyAsync(bcopy.p, b, (size_t)nn * nrhs * sizeof(double), hipMemcpyDeviceToDevice, stream));
        bb = bcopy.as<double>();
    }
    nebem_status worst = NEBEM_OK;
    nebem_solve_info agg = {0, 0.0};
    for (int64_t q = 0; q < nrhs; ++q) {
        nebem_solve_info ci;
        st = solve_mixed(A, a32.as<float>(), scale.as<double>(), dperm.as<int>(), nn, bb + q * n, sigma + q * n,
                         o.ir_tol, o.ir_max_iter, &ci, stream);
        if (st && st != NEBEM_ENOCONV) return st;
        if (st) worst = st;
        agg.ir_iters = ci.ir_iters > agg.ir_iters ? ci.ir_iters : agg.ir_iters;
        agg.rel_resid = ci.rel_resid > agg.rel_resid ? ci.rel_resid : agg.rel_resid;
    }
    if (info) *info = agg;
    NEBEM_HIP(hipStreamSynchronize(stream));
    return worst;
}

nebem_status nebem_solve_factored(const double *LU, const int32_t *ipiv, int64_t n, const double *b, int64_t nrhs,
                                  double *sigma, hipStream_t stream)
{
    if (n < 0 || n > 65536 * 4 || nrhs < 0 || nrhs > 4096) return fail(NEBEM_EINVAL, "solve_factored: bad sizes");
    if (n == 0 || nrhs == 0) return NEBEM_OK;
    if (!LU || !ipiv || !b || !sigma) return fail(NEBEM_EINVAL, "solve_factored: NULL argument");
    const int nn = (int)n;
    std::vector<int> hpiv(nn), perm;
    NEBEM_HIP(hipMemcpyAsync(hpiv.data(), ipiv, (size_t)nn * sizeof(int), hipMemcpyDeviceToHost, stream));
    NEBEM_HIP(hipStreamSynchronize(stream));
    for (int k = 0; k < nn; ++k)
        if (hpiv[k] < k || hpiv[k] >= nn) return fail(NEBEM_EINVAL, "solve_factored: ipiv is not a valid pivot list");
    pivots_to_perm(hpiv, perm);
    DevBuf dperm;
    NEBEM_HIP(dperm.alloc((size_t)nn * sizeof(int), stream));
    NEBEM_HIP(hipMemcpyAsync(dperm.p, perm.data(), (size_t)nn * sizeof(int), hipMemcpyHostToDevice, stream));
    nebem_status st = solve_fp64(LU, nn, dperm.as<int>(), b, (int)nrhs, sigma, stream);
    NEBEM_HIP(hipStreamSynchronize(stream));
    return st;
}

nebem_status nebem_norm1(const double *A, int64_t n, double *anorm, hipStream_t stream)
{
    if (n < 0 || n > 65536 * 4) return fail(NEBEM_EINVAL, "norm1: n out of range");
    if (!anorm || (n > 0 && !A)) return fail(NEBEM_EINVAL, "norm1: NULL argument");
    if (n == 0) {
        *anorm = 0.0;
        return NEBEM_OK;
    }
    return norm1_fp64(A, (int)n, anorm, stream);
}

nebem_status nebem_condest(const double *LU, const int32_t *ipiv, int64_t n, double anorm, double *kappa1,
                           hipStream_t stream)
{
    if (n < 0 || n > 65536 * 4) return fail(NEBEM_EINVAL, "condest: n out of range");
    if (!kappa1 || (n > 0 && (!LU || !ipiv))) return fail(NEBEM_EINVAL, "condest: NULL argument");
    if (!(anorm >= 0.0)) return fail(NEBEM_EINVAL, "condest: anorm must be >= 0");
    if (n == 0) {
        *kappa1 = 0.0;
        return NEBEM_OK;
    }
    const int nn = (int)n;
    std::vector<int> hpiv(nn), perm;
    NEBEM_HIP(hipMemcpyAsync(hpiv.data(), ipiv, (size_t)nn * sizeof(int), hipMemcpyDeviceToHost, stream));
    NEBEM_HIP(hipStreamSynchronize(stream));
    for (int k = 0; k < nn; ++k)
        if (hpiv[k] < k || hpiv[k] >= nn) return fail(NEBEM_EINVAL, "condest: ipiv is not a valid pivot list");
    pivots_to_perm(hpiv, perm);
    DevBuf dperm;
    NEBEM_HIP(dperm.alloc((size_t)nn * sizeof(int), stream));
    NEBEM_HIP(hipMemcpyAsync(dperm.p, perm.data(), (size_t)nn * sizeof(int), hipMemcpyHostToDevice, stream));
    return condest_fp64(LU, dperm.as<int>(), nn, anorm, kappa1, stream);
}

}  // extern "C"
