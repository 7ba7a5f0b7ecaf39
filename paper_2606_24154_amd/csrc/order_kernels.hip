// order_kernels.hip -- evaluation in spatial (Morton) order of the points.
//
// The field kernels give every lane one point and walk the elements in the
// same order for all lanes; a point's arithmetic does not depend on the other
// points of its wave, so the order in which points are packed into waves
// changes no bit of any result.  It does change how much work a wave does:
// the per-lane choice between the near and the far evaluation of an element
// copy (and, on the mixed path, among the far-field tiers) is a divergent
// branch, and a wave whose 64 points are scattered over the cell executes
// several of them for the same copy.  Sorting the points along a Morton curve
// of their bounding box packs neighbours into a wave, whose lanes then agree
// on the branch for nearly every copy.  Results are scattered back to the
// caller's order.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>

#include "nebem_internal.hpp"

namespace nebem {

constexpr int kOB = 256;         // threads per block of the helper kernels
constexpr int kBoxParts = 256;   // partial bounding boxes (first reduction pass)
constexpr int64_t kOrderMin = 4096;

// per-block bounding box of a strided share of the points (min / max are
// exact, so the result does not depend on the reduction order)
__global__ __launch_bounds__(kOB) void k_bbox_part(const double *__restrict__ px, const double *__restrict__ py,
                                                   const double *__restrict__ pz, int m, double *__restrict__ part)
{
    __shared__ double red[6][kOB];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * kOB + threadIdx.x; i < m; i += gridDim.x * kOB) {
        const double c[3] = {px[i], py[i], pz[i]};
        for (int k = 0; k < 3; ++k) {
            v[k] = fmin(v[k], c[k]);
            v[3 + k] = fmax(v[3 + k], c[k]);
        }
    }
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = kOB / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int k = 0; k < 6; ++k)
                red[k][threadIdx.x] = k < 3 ? fmin(red[k][threadIdx.x], red[k][threadIdx.x + h])
                                            : fmax(red[k][threadIdx.x], red[k][threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// 10-bit coordinate -> bits spread to every third position
__device__ __forceinline__ unsigned spread3(unsigned x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ unsigned quant10(double v, double lo, double sc)
{
    const double t = (v - lo) * sc;  // NaN coordinates fail both tests -> 0
    return t >= 1023.0 ? 1023u : (t > 0.0 ? (unsigned)t : 0u);
}

// keys[i] = Morton code of point i in the box (reduced from nparts partial
// boxes by every block: nparts x 6 doubles, L2-resident), idx[i] = i
__global__ __launch_bounds__(kOB) void k_keys(const double *__restrict__ px, const double *__restrict__ py,
                                              const double *__restrict__ pz, int m,
                                              const double *__restrict__ part, int nparts,
                                              unsigned *__restrict__ keys, int *__restrict__ idx)
{
    __shared__ double box[6];
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double b = k < 3 ? INFINITY : -INFINITY;
        for (int p = 0; p < nparts; ++p) b = k < 3 ? fmin(b, part[p * 6 + k]) : fmax(b, part[p * 6 + k]);
        box[k] = b;
    }
    __syncthreads();
    const int i = blockIdx.x * kOB + threadIdx.x;
    if (i >= m) return;
    unsigned q[3];
    const double c[3] = {px[i], py[i], pz[i]};
    for (int k = 0; k < 3; ++k) {
        const double ext = box[3 + k] - box[k];
        const double sc = (ext > 0.0 && ext < INFINITY) ? 1024.0 / ext : 0.0;
        q[k] = quant10(c[k], box[k], sc);
    }
    keys[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    idx[i] = i;
}

__global__ __launch_bounds__(kOB) void k_gather3(const double *__restrict__ px, const double *__restrict__ py,
                                                 const double *__restrict__ pz, const int *__restrict__ perm, int m,
                                                 double *__restrict__ sx, double *__restrict__ sy,
                                                 double *__restrict__ sz)
{
    const int k = blockIdx.x * kOB + threadIdx.x;
    if (k >= m) return;
    const int i = perm[k];
    sx[k] = px[i];
    sy[k] = py[i];
    sz[k] = pz[i];
}

// dst_j[perm[k]] = src[j * m + k] for every non-null destination j
__global__ __launch_bounds__(kOB) void k_scatter4(const double *__restrict__ src, const int *__restrict__ perm, int m,
                                                  double *__restrict__ d0, double *__restrict__ d1,
                                                  double *__restrict__ d2, double *__restrict__ d3)
{
    const int k = blockIdx.x * kOB + threadIdx.x;
    if (k >= m) return;
    const int i = perm[k];
    const size_t mm = (size_t)m;
    if (d0) d0[i] = src[k];
    if (d1) d1[i] = src[mm + k];
    if (d2) d2[i] = src[2 * mm + k];
    if (d3) d3[i] = src[3 * mm + k];
}

namespace {
// scratch of one sort: keys (in/out), identity indices, partial boxes, sort temp
struct SortLayout {
    size_t keys_in, keys_out, idx_in, part, sort, total;
    size_t sort_bytes;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

hipError_t sort_layout(int64_t m, SortLayout &L)
{
    size_t sort_bytes = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, sort_bytes, (const unsigned *)nullptr, (unsigned *)nullptr,
                                             (const int *)nullptr, (int *)nullptr, (int)m, 0u, 30u);
    if (e != hipSuccess) return e;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    L.keys_in = take(4 * (size_t)m);
    L.keys_out = take(4 * (size_t)m);
    L.idx_in = take(4 * (size_t)m);
    L.part = take(sizeof(double) * 6 * kBoxParts);
    L.sort = take(sort_bytes);
    L.sort_bytes = sort_bytes;
    L.total = off;
    return hipSuccess;
}
}  // namespace

bool eval_ordering_pays(int64_t m) { return m >= kOrderMin; }

size_t order_points_workspace(int64_t m)
{
    SortLayout L;
    if (sort_layout(m, L) != hipSuccess) return 0;
    return L.total;
}

hipError_t launch_order_points(const double *px, const double *py, const double *pz, int64_t m, double *sx,
                               double *sy, double *sz, int *perm, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    SortLayout L;
    hipError_t e = sort_layout(m, L);
    if (e != hipSuccess) return e;
    if (!ws || ws_bytes < L.total) return hipErrorInvalidValue;
    char *w = static_cast<char *>(ws);
    unsigned *keys_in = reinterpret_cast<unsigned *>(w + L.keys_in);
    unsigned *keys_out = reinterpret_cast<unsigned *>(w + L.keys_out);
    int *idx_in = reinterpret_cast<int *>(w + L.idx_in);
    double *part = reinterpret_cast<double *>(w + L.part);
    const int mi = (int)m;
    const unsigned g = (unsigned)((m + kOB - 1) / kOB);
    const int nparts = (int)std::min<int64_t>(kBoxParts, g);
    hipLaunchKernelGGL(k_bbox_part, dim3(nparts), dim3(kOB), 0, s, px, py, pz, mi, part);
    hipLaunchKernelGGL(k_keys, dim3(g), dim3(kOB), 0, s, px, py, pz, mi, part, nparts, keys_in, idx_in);
    size_t sort_bytes = L.sort_bytes;
    e = rocprim::radix_sort_pairs(w + L.sort, sort_bytes, keys_in, keys_out, idx_in, perm, mi, 0u, 30u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather3, dim3(g), dim3(kOB), 0, s, px, py, pz, perm, mi, sx, sy, sz);
    return hipGetLastError();
}

void launch_unorder4(const double *src, const int *perm, int64_t m, double *d0, double *d1, double *d2, double *d3,
                     hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_scatter4, dim3((unsigned)((m + kOB - 1) / kOB)), dim3(kOB), 0, s, src, perm, (int)m, d0, d1,
                       d2, d3);
}

// ------------------------------------------------------- evaluation driver
namespace {
constexpr size_t kPartBudget = size_t(512) << 20;  // preferred bytes of segment partial sums per chunk

struct EvalShape {
    SegPlan sp;
    int kc;           // columns per launch
    size_t part_pp;   // partial-sum bytes per point (0: one segment, no partials)
};

EvalShape eval_shape(int64_t n, const ImgArgs &img, int ncol)
{
    EvalShape sh;
    sh.sp = seg_plan(n, img);
    sh.kc = ncol < kMultiCols ? ncol : kMultiCols;
    sh.part_pp = sh.sp.nseg > 1 ? (size_t)32 * sh.kc * sh.sp.nseg : 0;
    return sh;
}

// workspace layout of one chunk of c points: [sort scratch | perm | sorted
// points | sorted results (kc columns)] when ordered, then the partial sums
struct ChunkLayout {
    bool ordered;
    size_t sort_ws, perm, pts, res, part, total;
};

bool chunk_layout(const EvalShape &sh, int64_t c, ChunkLayout &L)
{
    L.ordered = eval_ordering_pays(c);
    size_t off = 0;
    L.sort_ws = L.perm = L.pts = L.res = 0;
    if (L.ordered) {
        const size_t w = order_points_workspace(c);
        if (!w) return false;
        L.sort_ws = w;
        off = w;
        L.perm = off;
        off += align256(4 * (size_t)c);
        L.pts = off;
        off += align256(24 * (size_t)c);
        L.res = off;
        off += align256(32 * (size_t)sh.kc * (size_t)c);
    }
    L.part = off;
    off += align256(sh.part_pp * (size_t)c);
    L.total = off;
    return true;
}

int64_t preferred_chunk(const EvalShape &sh, int64_t m)
{
    int64_t c = m;
    if (sh.part_pp) {
        const int64_t lim = (int64_t)(kPartBudget / sh.part_pp) & ~(int64_t)255;
        c = std::min<int64_t>(m, std::max<int64_t>(lim, 256));
    }
    return c;
}

// one chunk of c points (unsorted input px.., outputs o.c[comp] + col * ostride)
void eval_chunk(const double *drec, const double *sigma, int64_t n, int ncol, const EvalShape &sh,
                const ImgArgs &img, int mixed, double near_factor, const double *px, const double *py,
                const double *pz, int64_t c, const OutCols &o, double *part, hipStream_t s)
{
    for (int c0 = 0; c0 < ncol; c0 += kMultiCols) {
        const int k = ncol - c0 < kMultiCols ? ncol - c0 : kMultiCols;
        const double *sg = sigma + (size_t)c0 * n;
        OutCols oc = o;
        for (int q = 0; q < 4; ++q) oc.c[q] = o.c[q] ? o.c[q] + (size_t)c0 * o.stride : nullptr;
        if (sh.sp.nseg == 1) {
            if (ncol == 1)
                launch_eval_seg(drec, sg, n, sh.sp, img, mixed, near_factor, px, py, pz, c, kKe, oc.c[0], oc.c[1],
                                oc.c[2], oc.c[3], 0, s);
            else
                launch_eval_multi_seg(drec, sg, n, n, k, sh.sp, img, mixed, near_factor, px, py, pz, c, kKe, oc, 0,
                                      s);
            continue;
        }
        // partials: column j, component q of segment y at part + y * 4 k c + (4 j + q) c
        const size_t cc = (size_t)c;
        OutCols pc = {{o.c[0] ? part : nullptr, o.c[1] ? part + cc : nullptr, o.c[2] ? part + 2 * cc : nullptr,
                       o.c[3] ? part + 3 * cc : nullptr},
                      (int64_t)(4 * cc)};
        const int64_t seg_stride = (int64_t)(4 * (size_t)k * cc);
        if (ncol == 1)
            launch_eval_seg(drec, sg, n, sh.sp, img, mixed, near_factor, px, py, pz, c, 1.0, pc.c[0], pc.c[1], pc.c[2],
                            pc.c[3], seg_stride, s);
        else
            launch_eval_multi_seg(drec, sg, n, n, k, sh.sp, img, mixed, near_factor, px, py, pz, c, 1.0, pc,
                                  seg_stride, s);
        launch_reduce_segments(part, sh.sp.nseg, k, c, seg_stride, oc, s);
    }
}
}  // namespace

size_t eval_workspace(int64_t n, const ImgArgs &img, int64_t m, int ncol)
{
    if (m <= 0 || ncol <= 0 || n <= 0) return 0;
    const EvalShape sh = eval_shape(n, img, ncol);
    ChunkLayout L;
    if (!chunk_layout(sh, preferred_chunk(sh, m), L)) return 0;
    return L.total;
}

size_t eval_workspace_min(int64_t n, const ImgArgs &img, int64_t m, int ncol)
{
    if (m <= 0 || ncol <= 0 || n <= 0) return 0;
    const EvalShape sh = eval_shape(n, img, ncol);
    ChunkLayout L;
    if (!chunk_layout(sh, std::min<int64_t>(m, 256), L)) return 0;
    return L.total;
}

hipError_t run_eval(const double *drec, const double *sigma, int64_t n, int ncol, const ImgArgs &img, int mixed,
                    double near_factor, const double *px, const double *py, const double *pz, int64_t m, double *phi,
                    double *ex, double *ey, double *ez, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (m <= 0 || ncol <= 0) return hipSuccess;
    const size_t mm = (size_t)m;
    if (n <= 0) {  // no elements: zero fields
        for (double *o : {phi, ex, ey, ez})
            if (o) {
                hipError_t e = hipMemsetAsync(o, 0, mm * (size_t)ncol * sizeof(double), s);
                if (e != hipSuccess) return e;
            }
        return hipSuccess;
    }
    const EvalShape sh = eval_shape(n, img, ncol);
    // the largest chunk (up to the preferred one) whose workspace fits
    int64_t c = preferred_chunk(sh, m);
    ChunkLayout L;
    for (;;) {
        if (!chunk_layout(sh, c, L)) return hipErrorInvalidValue;
        if (L.total <= ws_bytes || (L.total == 0)) break;
        if (c <= 256) return hipErrorInvalidValue;
        c = std::max<int64_t>(256, (c / 2) & ~(int64_t)255);
    }
    if (L.total > 0 && !ws) return hipErrorInvalidValue;
    // as many chunks as needed, of equal size (a short last chunk would be a
    // launch too small to fill the device)
    {
        const int64_t nch = (m + c - 1) / c;
        const int64_t even = ((m + nch - 1) / nch + 255) & ~(int64_t)255;
        if (even < c) c = even;
    }
    char *w = static_cast<char *>(ws);
    double *part = sh.part_pp ? reinterpret_cast<double *>(w + L.part) : nullptr;
    for (int64_t p0 = 0; p0 < m; p0 += c) {
        const int64_t cnt = std::min<int64_t>(c, m - p0);
        ChunkLayout Lc;
        if (!chunk_layout(sh, cnt, Lc) || Lc.total > ws_bytes) return hipErrorInvalidValue;
        if (!Lc.ordered) {
            OutCols o = {{phi ? phi + p0 : nullptr, ex ? ex + p0 : nullptr, ey ? ey + p0 : nullptr,
                          ez ? ez + p0 : nullptr},
                         m};
            eval_chunk(drec, sigma, n, ncol, sh, img, mixed, near_factor, px + p0, py + p0, pz + p0, cnt, o, part, s);
            continue;
        }
        const size_t cc = (size_t)cnt;
        int *perm = reinterpret_cast<int *>(w + Lc.perm);
        double *sp = reinterpret_cast<double *>(w + Lc.pts);
        double *so = reinterpret_cast<double *>(w + Lc.res);
        double *pc = sh.part_pp ? reinterpret_cast<double *>(w + Lc.part) : nullptr;
        hipError_t e = launch_order_points(px + p0, py + p0, pz + p0, cnt, sp, sp + cc, sp + 2 * cc, perm, ws,
                                           Lc.sort_ws, s);
        if (e != hipSuccess) return e;
        for (int c0 = 0; c0 < ncol; c0 += kMultiCols) {
            const int k = ncol - c0 < kMultiCols ? ncol - c0 : kMultiCols;
            // sorted results of column j of this column block: so + 4 j cnt (phi, ex, ey, ez)
            OutCols o = {{phi ? so : nullptr, ex ? so + cc : nullptr, ey ? so + 2 * cc : nullptr,
                          ez ? so + 3 * cc : nullptr},
                         (int64_t)(4 * cc)};
            eval_chunk(drec, sigma + (size_t)c0 * n, n, k, sh, img, mixed, near_factor, sp, sp + cc, sp + 2 * cc,
                       cnt, o, pc, s);
            for (int j = 0; j < k; ++j) {
                const size_t col = (size_t)(c0 + j) * mm + (size_t)p0;
                launch_unorder4(so + 4 * (size_t)j * cc, perm, cnt, phi ? phi + col : nullptr,
                                ex ? ex + col : nullptr, ey ? ey + col : nullptr, ez ? ez + col : nullptr, s);
            }
        }
    }
    return hipGetLastError();
}

}  // namespace nebem
