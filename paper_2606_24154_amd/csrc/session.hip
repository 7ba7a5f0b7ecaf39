// session.hip -- resident geometries (C-ABI nebem_session_*) and the dynamic
// space-charge step.
//
// A session holds, in device memory, everything the paper keeps resident
// between right-hand sides (Sec. 4.1): the derived element records, the
// influence matrix and its factors (the FP64 matrix plus its FP64 LU, or for
// the mixed path the equilibrated FP32 LU), the boundary values and the current
// surface charge densities.  nebem_spacecharge_step is one time step of the
// dynamic loop of Sec. 4.3 (Algorithm 4) with point charges (Sec. 4.2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "charge_internal.hpp"
#include "host_util.hpp"
#include "nebem_internal.hpp"
#include "session_internal.hpp"

using namespace nebem;

namespace nebem {

// sigma = A^-1 b with the session's factors
static nebem_status session_solve(nebem_session *s, const double *b, hipStream_t st)
{
    const int n = (int)s->n;
    if (s->opt.precision == NEBEM_FP64) {
        nebem_status e = solve_fp64(s->LU.as<double>(), n, s->perm.as<int>(), b, 1, s->sigma.as<double>(), st);
        if (e) return e;
        return refine_fp64(s->A.as<double>(), s->LU.as<double>(), s->perm.as<int>(), n, b, s->sigma.as<double>(),
                           kFp64RefineSteps, &s->last_info, st);
    }
    return solve_mixed(s->A.as<double>(), s->A32.as<float>(), s->scale.as<double>(), s->perm.as<int>(), n, b,
                       s->sigma.as<double>(), s->opt.ir_tol, s->opt.ir_max_iter, &s->last_info, st);
}

static nebem_status session_build(nebem_session *s, const nebem_panels *panels, hipStream_t st)
{
    const int64_t n = s->n;
    const int nn = (int)n;
    NEBEM_HIP(s->drec.ensure((size_t)n * R_STRIDE * sizeof(double)));
    {
        DevBuf tmp;
        nebem_status e = derive(panels, st, tmp);
        if (e) return e;
        NEBEM_HIP(hipMemcpyAsync(s->drec.p, tmp.p, (size_t)n * R_STRIDE * sizeof(double), hipMemcpyDeviceToDevice,
                                 st));
    }
    const bool mixed = s->opt.precision == NEBEM_MIXED;
    NEBEM_HIP(s->A.ensure((size_t)n * n * sizeof(double)));
    launch_assemble(s->drec.as<double>(), n, s->img, nullptr, nullptr, nullptr, s->A.as<double>(), st);
    NEBEM_HIP(hipGetLastError());
    NEBEM_HIP(s->ipiv.ensure((size_t)n * sizeof(int)));
    NEBEM_HIP(s->perm.ensure((size_t)n * sizeof(int)));
    std::vector<int> perm;
    nebem_status e;
    if (!mixed) {  // A stays unfactored for the refinement residuals
        NEBEM_HIP(s->LU.ensure((size_t)n * n * sizeof(double)));
        NEBEM_HIP(hipMemcpyAsync(s->LU.p, s->A.p, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, st));
        e = factor_fp64(s->LU.as<double>(), nn, s->ipiv.as<int>(), perm, st);
    } else {
        NEBEM_HIP(s->A32.ensure((size_t)n * n * sizeof(float)));
        NEBEM_HIP(s->scale.ensure((size_t)n * sizeof(double)));
        e = factor_mixed(s->A.as<double>(), nn, s->A32.as<float>(), s->scale.as<double>(), s->ipiv.as<int>(), perm,
                         st);
    }
    if (e) return e;
    NEBEM_HIP(hipMemcpyAsync(s->perm.p, perm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
    NEBEM_HIP(s->b0.ensure((size_t)n * sizeof(double)));
    NEBEM_HIP(s->sigma.ensure((size_t)n * sizeof(double)));
    NEBEM_HIP(s->rhs.ensure((size_t)n * sizeof(double)));
    launch_boundary_values(panels->bc, panels->value, n, s->b0.as<double>(), st);
    NEBEM_HIP(hipGetLastError());
    e = session_solve(s, s->b0.as<double>(), st);
    NEBEM_HIP(hipStreamSynchronize(st));  // perm (host) must outlive its copy
    return e;
}

// Evaluation over the resident geometry through the evaluation driver, with
// the session's own workspace (grown to the driver's preferred size).
static nebem_status session_eval_points(nebem_session *s, const double *px, const double *py, const double *pz,
                                        int64_t m, double *phi, double *ex, double *ey, double *ez, hipStream_t st)
{
    const int mixed = s->opt.precision == NEBEM_MIXED;
    const size_t wb = eval_workspace(s->n, s->img, m, 1);
    if (wb) NEBEM_HIP(s->ows.ensure(wb));
    NEBEM_HIP(run_eval(s->drec.as<double>(), s->sigma.as<double>(), s->n, 1, s->img, mixed, s->opt.near_factor, px,
                       py, pz, m, phi, ex, ey, ez, s->ows.p, s->ows.bytes, st));
    return NEBEM_OK;
}

// Algorithm 4's UpdateFields decision: the fixed schedule, or with
// sc_threshold >= 0 the charges' magnitude sum |q| against the threshold
// (partial sums on the device, added on the host in index order).
static nebem_status resolve_due(nebem_session *s, int step, const double *q, int64_t nq, hipStream_t st, bool &due)
{
    if (s->opt.sc_threshold < 0.0) {
        due = step % s->opt.sc_resolve_every == 0;
        return NEBEM_OK;
    }
    double total = 0.0;
    if (nq > 0) {
        NEBEM_HIP(s->absq.ensure(kAbsParts * sizeof(double)));
        const int np = launch_abs_sum(q, nq, s->absq.as<double>(), st);
        NEBEM_HIP(hipGetLastError());
        double h[kAbsParts];
        NEBEM_HIP(hipMemcpyAsync(h, s->absq.p, np * sizeof(double), hipMemcpyDeviceToHost, st));
        NEBEM_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < np; ++k) total += h[k];
    }
    due = total > s->opt.sc_threshold;
    return NEBEM_OK;
}

// The session's FastVolume map (Algorithm 4's CreateFastVolPF): panels with
// the current sigma at every node, plus the charges' own field (point
// charges, or lines when `lines` is set), interleaved into the caller's
// buffer.
static nebem_status refresh_fastvol(nebem_session *s, const double *qx, const double *qy, const double *qz,
                                    const double *q, int64_t nq, const double *lines, int64_t nl, hipStream_t st)
{
    if (!s->fv_kind) return NEBEM_OK;
    const size_t nn = (size_t)s->fv_nodes;
    NEBEM_HIP(s->fv_tmp.ensure(7 * nn * sizeof(double)));
    double *t = s->fv_tmp.as<double>();
    if (s->fv_kind == 1)
        launch_grid_nodes(s->fv_grid, t, t + nn, t + 2 * nn, st);
    else
        launch_axes_nodes(s->fv_axes, t, t + nn, t + 2 * nn, st);
    NEBEM_HIP(hipGetLastError());
    nebem_status e = session_eval_points(s, t, t + nn, t + 2 * nn, (int64_t)nn, t + 3 * nn, t + 4 * nn, t + 5 * nn,
                                         t + 6 * nn, st);
    if (e) return e;
    if (lines && nl > 0) {
        NEBEM_HIP(s->lf.ensure(4 * nn * sizeof(double)));
        double *f = s->lf.as<double>();
        launch_line_field(lines, nl, t, t + nn, t + 2 * nn, (int64_t)nn, f, f + nn, f + 2 * nn, f + 3 * nn, st);
        launch_add4(f, (int64_t)nn, t + 3 * nn, t + 4 * nn, t + 5 * nn, t + 6 * nn, st);
    } else if (!lines && nq > 0) {
        launch_point_field(t, t + nn, t + 2 * nn, (int64_t)nn, qx, qy, qz, q, nq, t + 3 * nn, t + 4 * nn, t + 5 * nn,
                           t + 6 * nn, st);
    }
    launch_interleave4(t + 3 * nn, t + 4 * nn, t + 5 * nn, t + 6 * nn, (int64_t)nn, s->fv_values, st);
    NEBEM_HIP(hipGetLastError());
    return NEBEM_OK;
}

// ---- allocation-free evaluation
// Scratch of nebem_session_eval_noalloc: a file-scope device array, one
// copy per GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address): each device's address is taken once with
// hipGetSymbolAddress, with that device current, and kept.
constexpr size_t kNoAllocScratch = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratch];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;

static nebem_status scratch_address(void **out)
{
    int dev = 0;
    NEBEM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return NEBEM_OK;
}

}  // namespace nebem

extern "C" {

nebem_status nebem_session_create(const nebem_panels *panels, const nebem_images *images, const nebem_options *opt,
                                  hipStream_t stream, nebem_session **out)
{
    if (!out) return fail(NEBEM_EINVAL, "session_create: NULL output");
    *out = nullptr;
    nebem_status st = check_panels(panels);
    if (st) return st;
    if (panels->n == 0) return fail(NEBEM_EINVAL, "session_create: no panels");
    if (panels->n > 65536 * 4) return fail(NEBEM_EINVAL, "session_create: too many panels");
    nebem_options o;
    if (opt)
        o = *opt;
    else
        nebem_default_options(&o);
    if ((st = check_options(o))) return st;
    if (o.sc_resolve_every < 1 || !(o.sc_dt >= 0.0) || !(o.sc_mobility >= 0.0) || !std::isfinite(o.sc_threshold))
        return fail(NEBEM_EINVAL, "session_create: bad space-charge options");
    nebem_session *s = new (std::nothrow) nebem_session;
    if (!s) return fail(NEBEM_ENOMEM, "session_create: host allocation failed");
    s->n = panels->n;
    s->opt = o;
    if ((st = make_img_args(images, &s->img))) {
        delete s;
        return st;
    }
    s->img_count = (double)s->img.nref * (2 * s->img.n1 + 1) * (2 * s->img.n2 + 1);
    st = session_build(s, panels, stream);
    if (st && st != NEBEM_ENOCONV) {
        (void)hipStreamSynchronize(stream);
        delete s;
        return st;
    }
    *out = s;
    return st;
}

void nebem_session_destroy(nebem_session *s) { delete s; }

int64_t nebem_session_n(const nebem_session *s) { return s ? s->n : 0; }

const double *nebem_session_sigma(const nebem_session *s) { return s ? s->sigma.as<double>() : nullptr; }

nebem_status nebem_session_solve(nebem_session *s, const double *b, nebem_solve_info *info, hipStream_t stream)
{
    if (!s || !b) return fail(NEBEM_EINVAL, "session_solve: NULL argument");
    nebem_status st = session_solve(s, b, stream);
    if (info) *info = s->last_info;
    if (!st) NEBEM_HIP(hipStreamSynchronize(stream));
    return st;
}

nebem_status nebem_session_condest(nebem_session *s, double *kappa1, hipStream_t stream)
{
    if (!s || !kappa1) return fail(NEBEM_EINVAL, "session_condest: NULL argument");
    if (s->opt.precision != NEBEM_FP64) return fail(NEBEM_EINVAL, "session_condest: needs an FP64 session");
    const int n = (int)s->n;
    if (n == 0) {
        *kappa1 = 0.0;
        return NEBEM_OK;
    }
    double anorm = 0.0;
    nebem_status st = norm1_fp64(s->A.as<double>(), n, &anorm, stream);
    if (st) return st;
    return condest_fp64(s->LU.as<double>(), s->perm.as<int>(), n, anorm, kappa1, stream);
}

nebem_status nebem_session_eval(nebem_session *s, const double *px, const double *py, const double *pz, int64_t m,
                                double *phi, double *ex, double *ey, double *ez, hipStream_t stream)
{
    if (!s) return fail(NEBEM_EINVAL, "session_eval: NULL session");
    if (m < 0 || m > (int64_t)INT32_MAX - 256) return fail(NEBEM_EINVAL, "session_eval: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!px || !py || !pz) return fail(NEBEM_EINVAL, "session_eval: NULL point array");
    return session_eval_points(s, px, py, pz, m, phi, ex, ey, ez, stream);
}

nebem_status nebem_session_fastvol(nebem_session *s, const nebem_grid *grid, const nebem_axes *axes, double *values,
                                   hipStream_t stream)
{
    if (!s) return fail(NEBEM_EINVAL, "session_fastvol: NULL session");
    if (!grid && !axes) {
        s->fv_kind = 0;
        s->fv_values = nullptr;
        return NEBEM_OK;
    }
    if (grid && axes) return fail(NEBEM_EINVAL, "session_fastvol: give a regular grid or graded axes, not both");
    if (!values) return fail(NEBEM_EINVAL, "session_fastvol: NULL values");
    if ((uintptr_t)values % 16) return fail(NEBEM_EINVAL, "session_fastvol: values must be 16-byte aligned");
    int64_t nn = 1;
    if (grid) {
        GridArgs g;
        for (int a = 0; a < 3; ++a) {
            if (grid->n[a] < 2 || !(grid->step[a] > 0.0) || !std::isfinite(grid->step[a]) ||
                !std::isfinite(grid->origin[a]))
                return fail(NEBEM_EINVAL, "session_fastvol: bad regular grid");
            g.origin[a] = grid->origin[a];
            g.step[a] = grid->step[a];
            g.inv_step[a] = 1.0 / grid->step[a];
            g.n[a] = grid->n[a];
            nn *= grid->n[a];
            if (nn > (int64_t)INT32_MAX - 256) return fail(NEBEM_EINVAL, "session_fastvol: too many nodes");
        }
        s->fv_grid = g;
        s->fv_kind = 1;
    } else {
        AxesArgs g;
        if (!axes->x || !axes->y || !axes->z) return fail(NEBEM_EINVAL, "session_fastvol: NULL axis");
        g.ax[0] = axes->x;
        g.ax[1] = axes->y;
        g.ax[2] = axes->z;
        for (int a = 0; a < 3; ++a) {
            if (axes->n[a] < 2) return fail(NEBEM_EINVAL, "session_fastvol: fewer than 2 nodes on an axis");
            g.n[a] = axes->n[a];
            nn *= axes->n[a];
            if (nn > (int64_t)INT32_MAX - 256) return fail(NEBEM_EINVAL, "session_fastvol: too many nodes");
        }
        NEBEM_HIP(s->absq.ensure(kAbsParts * sizeof(double)));
        int *bad = reinterpret_cast<int *>(s->absq.p);
        NEBEM_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
        launch_axes_check(g, bad, stream);
        NEBEM_HIP(hipGetLastError());
        int hbad = 0;
        NEBEM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
        NEBEM_HIP(hipStreamSynchronize(stream));
        if (hbad) return fail(NEBEM_EINVAL, "session_fastvol: an axis is not strictly increasing and finite");
        s->fv_axes = g;
        s->fv_kind = 2;
    }
    s->fv_values = values;
    s->fv_nodes = nn;
    nebem_status st = refresh_fastvol(s, nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0, stream);
    if (st) {
        s->fv_kind = 0;
        return st;
    }
    NEBEM_HIP(hipStreamSynchronize(stream));
    return NEBEM_OK;
}

nebem_status nebem_session_eval_noalloc(nebem_session *s, const double *px, const double *py, const double *pz,
                                        int64_t m, double *phi, double *ex, double *ey, double *ez,
                                        hipStream_t stream)
{
    if (!s) return fail(NEBEM_EINVAL, "session_eval_noalloc: NULL session");
    if (m < 0 || m > (int64_t)INT32_MAX - 256) return fail(NEBEM_EINVAL, "session_eval_noalloc: m out of range");
    if (m == 0) return NEBEM_OK;
    if (!px || !py || !pz) return fail(NEBEM_EINVAL, "session_eval_noalloc: NULL point array");
    if (eval_workspace_min(s->n, s->img, m, 1) > kNoAllocScratch)
        return fail(NEBEM_EINVAL, "session_eval_noalloc: the evaluation needs more than the " +
                                      std::to_string(kNoAllocScratch >> 20) + " MiB scratch");
    void *ws = nullptr;
    nebem_status st = scratch_address(&ws);
    if (st) return st;
    // the driver takes point chunks whose workspace fits the scratch; its
    // results do not depend on the chunking
    NEBEM_HIP(run_eval(s->drec.as<double>(), s->sigma.as<double>(), s->n, 1, s->img,
                       s->opt.precision == NEBEM_MIXED, s->opt.near_factor, px, py, pz, m, phi, ex, ey, ez, ws,
                       kNoAllocScratch, stream));
    return NEBEM_OK;
}

nebem_status nebem_spacecharge_step(nebem_session *s, double *qx, double *qy, double *qz, const double *q, int64_t nq,
                                    int32_t step_index, double *ex, double *ey, double *ez, hipStream_t stream)
{
    if (!s) return fail(NEBEM_EINVAL, "spacecharge_step: NULL session");
    if (nq < 0 || nq > (int64_t)INT32_MAX - 256) return fail(NEBEM_EINVAL, "spacecharge_step: nq out of range");
    if (step_index < 0) return fail(NEBEM_EINVAL, "spacecharge_step: negative step index");
    if (nq > 0 && (!qx || !qy || !qz || !q)) return fail(NEBEM_EINVAL, "spacecharge_step: NULL charge array");
    if ((ex == nullptr) != (ey == nullptr) || (ex == nullptr) != (ez == nullptr))
        return fail(NEBEM_EINVAL, "spacecharge_step: field arrays must be all NULL or all set");
    const int64_t n = s->n;
    nebem_status st = NEBEM_OK;
    bool due = false;
    if ((st = resolve_due(s, step_index, q, nq, stream, due))) return st;
    if (due) {
        const int nchunk = charge_rhs_chunks(n, nq);
        NEBEM_HIP(s->part.ensure((size_t)nchunk * n * sizeof(double)));
        launch_charge_rhs(s->drec.as<double>(), n, qx, qy, qz, q, nq, s->b0.as<double>(), s->part.as<double>(), nchunk,
                          s->rhs.as<double>(), stream);
        NEBEM_HIP(hipGetLastError());
        st = session_solve(s, s->rhs.as<double>(), stream);
        if (st && st != NEBEM_ENOCONV) return st;
        const nebem_status sf = refresh_fastvol(s, qx, qy, qz, q, nq, nullptr, 0, stream);
        if (sf) return sf;
    }
    if (nq == 0) return st;
    if (!ex) {
        NEBEM_HIP(s->eb.ensure((size_t)3 * nq * sizeof(double)));
        ex = s->eb.as<double>();
        ey = ex + nq;
        ez = ey + nq;
    }
    {
        const nebem_status se = session_eval_points(s, qx, qy, qz, nq, nullptr, ex, ey, ez, stream);
        if (se) return se;
    }
    {
        const size_t wb = coulomb_workspace(nq);
        if (!wb) return fail(NEBEM_EDEVICE, "spacecharge_step: workspace query failed");
        NEBEM_HIP(s->cws.ensure(wb));
        NEBEM_HIP(launch_coulomb(qx, qy, qz, q, nq, ex, ey, ez, s->cws.p, s->cws.bytes, stream));
    }
    launch_euler(qx, qy, qz, q, ex, ey, ez, nq, s->opt.sc_mobility * s->opt.sc_dt, stream);
    NEBEM_HIP(hipGetLastError());
    return st;
}

nebem_status nebem_spacecharge_step_lines(nebem_session *s, double *qx, double *qy, double *qz, const double *q,
                                          int64_t nq, int32_t step_index, const nebem_grid *vox, int32_t placement,
                                          double *ex, double *ey, double *ez, int64_t *nlines, hipStream_t stream)
{
    if (nlines) *nlines = 0;
    if (!s) return fail(NEBEM_EINVAL, "spacecharge_step_lines: NULL session");
    if (nq < 0 || nq > (int64_t)INT32_MAX - 256) return fail(NEBEM_EINVAL, "spacecharge_step_lines: nq out of range");
    if (step_index < 0) return fail(NEBEM_EINVAL, "spacecharge_step_lines: negative step index");
    if (nq > 0 && (!qx || !qy || !qz || !q)) return fail(NEBEM_EINVAL, "spacecharge_step_lines: NULL charge array");
    if ((ex == nullptr) != (ey == nullptr) || (ex == nullptr) != (ez == nullptr))
        return fail(NEBEM_EINVAL, "spacecharge_step_lines: field arrays must be all NULL or all set");
    if (placement != NEBEM_LINE_CENTRE && placement != NEBEM_LINE_WEIGHTED)
        return fail(NEBEM_EINVAL, "spacecharge_step_lines: unknown line placement");
    GridArgs g;
    nebem_status st = voxel_grid_args(vox, g);
    if (st) return st;
    const int64_t n = s->n;
    // 1. the charges as line charges (at most one per occupied voxel); the
    // workspace keeps the charges sorted by voxel for step 3
    int64_t nl = 0, outside = 0;
    if (nq > 0) {
        const int64_t nvox = (int64_t)g.n[0] * g.n[1] * g.n[2];
        const int64_t cap = nq < nvox ? nq : nvox;
        const size_t wb = voxel_workspace((int)nq);
        if (!wb) return fail(NEBEM_EDEVICE, "spacecharge_step_lines: workspace query failed");
        NEBEM_HIP(s->vws.ensure(wb));
        NEBEM_HIP(s->lines.ensure((size_t)cap * 7 * sizeof(double)));
        NEBEM_HIP(voxel_lines(qx, qy, qz, q, (int)nq, g, placement == NEBEM_LINE_WEIGHTED, s->lines.as<double>(),
                              cap, &nl, &outside, s->vws.p, s->vws.bytes, stream));
    }
    if (nlines) *nlines = nl;
    const double *lines = s->lines.as<double>();
    // 2. re-solve with the lines' share on the right-hand side
    bool due = false;
    if ((st = resolve_due(s, step_index, q, nq, stream, due))) return st;
    if (due) {
        NEBEM_HIP(s->part.ensure((size_t)7 * n * sizeof(double)));
        launch_line_rhs(s->drec.as<double>(), n, lines, nl, s->b0.as<double>(), s->part.as<double>(),
                        s->rhs.as<double>(), stream);
        NEBEM_HIP(hipGetLastError());
        st = session_solve(s, s->rhs.as<double>(), stream);
        if (st && st != NEBEM_ENOCONV) return st;
        const nebem_status sf = refresh_fastvol(s, qx, qy, qz, q, nq, lines, nl, stream);
        if (sf) return sf;
    }
    if (nq == 0) return st;
    if (!ex) {
        NEBEM_HIP(s->eb.ensure((size_t)3 * nq * sizeof(double)));
        ex = s->eb.as<double>();
        ey = ex + nq;
        ez = ey + nq;
    }
    // 3. E at the charges: panels + far lines + near charges, then the move
    {
        const nebem_status se = session_eval_points(s, qx, qy, qz, nq, nullptr, ex, ey, ez, stream);
        if (se) return se;
    }
    NEBEM_HIP(s->lf.ensure((size_t)4 * nq * sizeof(double)));
    double *t = s->lf.as<double>();
    launch_line_field_at_charges(lines, nl, s->vws.p, g, qx, qy, qz, q, (int)nq, t + nq, t + 2 * nq, t + 3 * nq,
                                 stream);
    launch_add4(t, nq, nullptr, ex, ey, ez, stream);
    launch_euler(qx, qy, qz, q, ex, ey, ez, nq, s->opt.sc_mobility * s->opt.sc_dt, stream);
    NEBEM_HIP(hipGetLastError());
    return st;
}

}  // extern "C"
