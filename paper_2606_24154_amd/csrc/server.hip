// server.hip -- continuous-batching field-evaluation service over resident
// geometries (C-ABI nebem_server_*).
//
// Clients (e.g. particle-drift loops, which in the paper query potential and
// field at millions of points, Sec. 3) submit batches of points on one of the
// server's resident sessions.  A worker thread runs the scheduling loop:
//   1. admission: queued requests enter, in arrival order, while their
//      staging (points, results, permutation and per-segment partial sums:
//      8 + 4 nseg doubles per point) fits into the device arena of
//      hbm_budget bytes.  A request that does not fit blocks the head of
//      the line; behind it, small requests (at most 1/64 of the arena) that
//      fit are admitted past it, placed at the arena's top end so that the
//      space freed below stays in one piece, at most kMaxBypass of them per
//      blocked head (so the head waits for a bounded number of them).
//      At most max_large requests of large_interactions or more are active
//      at once (by default one: first come first served among them, the
//      smaller ones sharing the device with them), so that the largest
//      requests do not all slow each other down.
//      Admitted points are copied in and, for requests of 4096 points or
//      more, sorted into Morton order on the device (so that the lanes of a
//      work item share the near/far branches; each lane's arithmetic is
//      unchanged);
//   2. batching: the active requests are cut into work items of 64 points x
//      one segment of the geometry's elements (each geometry's element range
//      is split into a fixed number of segments of about kSegWork
//      interactions per point, so that one heavy point is not a long serial
//      chain in a single lane), taken round-robin (one item per request per
//      round) until the iteration's interaction budget is used; items of
//      different requests and geometries go into ONE launch;
//   3. completion: a request whose items are all done has its segment
//      partial sums reduced in a fixed order (and scattered back to the
//      submission order if sorted), its results copied back to the
//      caller's host arrays, its arena space freed and its waiter woken; new
//      requests are admitted on the next iteration.
// Launches alternate between two streams, and the worker builds and issues
// launch L before it waits for launch L - 1: the device always holds the
// next launch, so the host's work between launches (completions, copies,
// admission, the next list) is hidden, and launch L's workgroups fill the
// slots that launch L - 1's last, uneven round leaves idle.  Admission
// work (point copies and sorts) runs on a third stream that each launch
// waits for.
// Each point's partial sums and their reduction have a fixed order that does
// not depend on the other requests, so a request's results are identical
// whether it runs alone or in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "host_util.hpp"
#include "nebem_internal.hpp"
#include "server_admission.hpp"
#include "session_internal.hpp"

namespace nebem {

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t id = 0;
    int geom = 0;
    int64_t m = 0;
    const double *hx = nullptr, *hy = nullptr, *hz = nullptr;
    double *hphi = nullptr, *hex = nullptr, *hey = nullptr, *hez = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t off = 0, bytes = 0;  // arena placement
    int nseg = 1;               // element segments of its geometry
    int64_t nitems = 0;         // 64-point chunks x segments
    int64_t next = 0;           // first item not yet scheduled
    int64_t infl[2] = {0, 0};   // items in the launch on stream 0 / 1 not yet retired
    int64_t done_items = 0;
    int status = NEBEM_OK;
    bool ordered = false;       // points sorted into Morton order on admission
    bool large = false;         // at least large_interactions of work
    bool waited = false;        // a nebem_server_wait call holds its ticket
    bool finished = false;
};

}  // namespace nebem

struct nebem_server {
    int device = 0;
    nebem_server_options opt;
    std::vector<nebem_session *> geoms;
    std::vector<int64_t> geom_n;
    std::vector<int> geom_nseg;   // element segments per geometry
    std::vector<int> geom_segsz;  // elements per segment (last may be shorter)
    int mixed = 0;
    double near_factor = 4.0;
    hipStream_t stream = nullptr;            // admission: point copies and sorts
    hipStream_t lst[2] = {nullptr, nullptr};  // item launches, alternating
    hipEvent_t ev_adm = nullptr, ev_launch[2] = {nullptr, nullptr};
    void *arena_dev = nullptr;
    nebem::Arena arena;
    nebem::ImgArgs *imgs_dev = nullptr;
    nebem::WorkItem *items_dev = nullptr;   // 2 x items_cap: one list per launch stream
    nebem::WorkItem *items_host = nullptr;  // pinned, 2 x items_cap
    void *sort_ws = nullptr;                // scratch of the point sort (grown on demand)
    size_t sort_ws_bytes = 0;
    int items_cap = 0;
    int round_items = 1;  // work items (waves) the device runs at once
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<nebem::Request *> queue;
    std::vector<nebem::Request *> active;
    nebem::AdmitState adm;
    std::map<int64_t, nebem::Request *> all;
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // statistics
    int64_t launches = 0, points_done = 0;
    double interactions_done = 0, busy_s = 0;
    std::string worker_error;
};

using namespace nebem;

namespace nebem {

static void admit_locked(nebem_server *s)
{
    admit(s->queue, s->arena, s->adm, s->opt.max_large, [&](Request *r) {
        r->t_admit = now_s();
        s->active.push_back(r);
    });
}

// device addresses of a request's staging: columns 0-2 points (sorted if
// ordered), 3-6 results, 7 the permutation (int32), then nseg x 4 columns of
// segment partial sums
static inline double *stage(nebem_server *s, const Request *r, int k)
{
    return reinterpret_cast<double *>(static_cast<char *>(s->arena_dev) + r->off) + (size_t)k * r->m;
}

static void worker_main(nebem_server *s)
{
    (void)hipSetDevice(s->device);
    std::vector<Request *> fresh;
    int64_t nlaunch = 0;     // launches issued
    int pend = -1;           // stream of the launch in flight, -1 if none
    bool adm_event = false;  // ev_adm recorded at least once
    double t_busy = 0.0;     // start of the current stretch with a launch in flight
    // statistics gathered outside the lock, added to the server's under it
    double d_inter = 0.0, d_busy = 0.0;
    int64_t d_launches = 0;
    for (;;) {
        std::vector<Request *> act;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (pend < 0)
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
            if (s->stop && s->queue.empty() && s->active.empty() && pend < 0) return;
            const size_t before = s->active.size();
            admit_locked(s);
            fresh.assign(s->active.begin() + before, s->active.end());
            act = s->active;
        }
        const int cur = (int)(nlaunch & 1);
        // copy the new requests' points in; large ones land in the result
        // columns and are sorted into the point columns
        for (Request *r : fresh) {
            const size_t b = (size_t)r->m * sizeof(double);
            const int c0 = r->ordered ? 3 : 0;
            hipError_t e = hipMemcpyAsync(stage(s, r, c0), r->hx, b, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(stage(s, r, c0 + 1), r->hy, b, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(stage(s, r, c0 + 2), r->hz, b, hipMemcpyHostToDevice, s->stream);
            if (e == hipSuccess && r->ordered) {
                const size_t wb = order_points_workspace(r->m);
                if (wb == 0) e = hipErrorInvalidValue;
                if (e == hipSuccess && wb > s->sort_ws_bytes) {
                    if (s->sort_ws) e = hipStreamSynchronize(s->stream);
                    if (e == hipSuccess && s->sort_ws) e = hipFree(s->sort_ws);
                    s->sort_ws = nullptr;
                    s->sort_ws_bytes = 0;
                    if (e == hipSuccess) e = hipMalloc(&s->sort_ws, wb);
                    if (e == hipSuccess) s->sort_ws_bytes = wb;
                }
                if (e == hipSuccess)
                    e = launch_order_points(stage(s, r, 3), stage(s, r, 4), stage(s, r, 5), r->m, stage(s, r, 0),
                                            stage(s, r, 1), stage(s, r, 2), reinterpret_cast<int *>(stage(s, r, 7)),
                                            s->sort_ws, s->sort_ws_bytes, s->stream);
            }
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->worker_error = hipGetErrorString(e);
                r->status = NEBEM_EDEVICE;
            }
        }
        if (!fresh.empty() && hipEventRecord(s->ev_adm, s->stream) == hipSuccess) adm_event = true;
        // build the work list: round-robin, one item per request per round,
        // until the iteration's budget is used and the list fills whole
        // rounds of the device's work-item slots (an item is one wave, and a
        // launch whose last round is part-filled leaves CUs idle at its end).
        // This stream's previous list (launch nlaunch - 2) has completed.
        WorkItem *items_host = s->items_host + (size_t)cur * s->items_cap;
        WorkItem *items_dev = s->items_dev + (size_t)cur * s->items_cap;
        int nitems = 0;
        double budget = s->opt.batch_interactions;
        bool progress = true;
        auto more = [&] { return budget > 0.0 || nitems % s->round_items != 0; };
        while (progress && more() && nitems < s->items_cap) {
            progress = false;
            for (Request *r : act) {
                if (r->status != NEBEM_OK || r->next >= r->nitems || nitems >= s->items_cap) continue;
                const nebem_session *g = s->geoms[r->geom];
                const int64_t chunk = r->next / r->nseg;
                const int seg = (int)(r->next % r->nseg);
                const int64_t p0 = chunk * 64;
                const int cnt = (int)std::min<int64_t>(64, r->m - p0);
                const int e0 = seg * s->geom_segsz[r->geom];
                const int ne = (int)std::min<int64_t>(s->geom_segsz[r->geom], g->n - e0);
                WorkItem &w = items_host[nitems++];
                w.drec = g->drec.as<double>() + (size_t)e0 * R_STRIDE;
                w.sigma = g->sigma.as<double>() + e0;
                w.n = ne;
                w.geom = r->geom;
                w.count = cnt;
                w.pad = 0;
                w.px = stage(s, r, 0) + p0;
                w.py = stage(s, r, 1) + p0;
                w.pz = stage(s, r, 2) + p0;
                w.phi = stage(s, r, 8 + 4 * seg) + p0;
                w.ex = stage(s, r, 9 + 4 * seg) + p0;
                w.ey = stage(s, r, 10 + 4 * seg) + p0;
                w.ez = stage(s, r, 11 + 4 * seg) + p0;
                r->next += 1;
                r->infl[cur] += 1;
                const double work = (double)ne * g->img_count * cnt;
                budget -= work;
                d_inter += work;
                progress = true;
                if (!more()) break;
            }
        }
        bool launched = false;
        if (nitems > 0) {
            hipError_t e = adm_event ? hipStreamWaitEvent(s->lst[cur], s->ev_adm, 0) : hipSuccess;
            if (e == hipSuccess)
                e = hipMemcpyAsync(items_dev, items_host, (size_t)nitems * sizeof(WorkItem), hipMemcpyHostToDevice,
                                   s->lst[cur]);
            if (e == hipSuccess) {
                launch_eval_items(items_dev, nitems, s->imgs_dev, s->mixed, s->near_factor, s->lst[cur]);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(s->ev_launch[cur], s->lst[cur]);
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->worker_error = hipGetErrorString(e);
                for (Request *r : act) r->status = NEBEM_EDEVICE;
            }
            if (pend < 0) t_busy = now_s();
            launched = true;
            ++nlaunch;
            ++d_launches;
        }
        // retire the previous launch: its requests whose items are all done
        // (or that failed and have nothing in flight) get their segments
        // reduced, results copied back, arena space freed
        std::vector<Request *> done;
        if (pend >= 0) {
            (void)hipEventSynchronize(s->ev_launch[pend]);
            for (Request *r : act) {
                r->done_items += r->infl[pend];
                r->infl[pend] = 0;
            }
        }
        for (Request *r : act)
            if (r->done_items >= r->nitems || (r->status != NEBEM_OK && r->infl[0] == 0 && r->infl[1] == 0))
                done.push_back(r);
        // results of sorted requests end in the first partial-sum columns, in
        // submission order
        const int rs = pend >= 0 ? pend : cur;  // a stream with nothing of these requests ahead
        for (Request *r : done)
            if (r->status == NEBEM_OK) {
                const OutCols out = {{stage(s, r, 3), stage(s, r, 4), stage(s, r, 5), stage(s, r, 6)}, r->m};
                launch_reduce_segments(stage(s, r, 8), r->nseg, 1, r->m, 4 * r->m, out, s->lst[rs]);
                if (r->ordered)
                    launch_unorder4(stage(s, r, 3), reinterpret_cast<const int *>(stage(s, r, 7)), r->m,
                                    stage(s, r, 8), stage(s, r, 9), stage(s, r, 10), stage(s, r, 11), s->lst[rs]);
            }
        if (!done.empty()) (void)hipStreamSynchronize(s->lst[rs]);
        if (!launched && pend >= 0) d_busy += now_s() - t_busy;
        pend = launched ? cur : -1;
        for (Request *r : done) {
            if (r->status == NEBEM_OK) {
                const size_t b = (size_t)r->m * sizeof(double);
                double *dst[4] = {r->hphi, r->hex, r->hey, r->hez};
                for (int k = 0; k < 4; ++k)
                    if (dst[k] && hipMemcpy(dst[k], stage(s, r, (r->ordered ? 8 : 3) + k), b,
                                            hipMemcpyDeviceToHost) != hipSuccess)
                        r->status = NEBEM_EDEVICE;
            }
            r->t_done = now_s();
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->interactions_done += d_inter;
            s->busy_s += d_busy;
            s->launches += d_launches;
            d_inter = d_busy = 0.0;
            d_launches = 0;
            for (Request *r : done) {
                s->arena.release(r->off, r->bytes);
                if (r->large) --s->adm.active_large;
                s->active.erase(std::find(s->active.begin(), s->active.end(), r));
                s->points_done += r->m;
                r->finished = true;
            }
        }
        if (!done.empty()) s->cv_done.notify_all();
    }
}

}  // namespace nebem

extern "C" {

void nebem_server_default_options(nebem_server_options *o)
{
    if (!o) return;
    o->hbm_budget = (int64_t)2 << 30;
    o->batch_interactions = 1e10;
    o->max_items = 65536;
    o->large_interactions = 1e11;
    o->max_large = 1;
}

nebem_status nebem_server_create(nebem_session *const *sessions, int32_t nsessions, const nebem_server_options *opt,
                                 nebem_server **out)
{
    if (!out) return fail(NEBEM_EINVAL, "server_create: NULL output");
    *out = nullptr;
    if (!sessions || nsessions < 1 || nsessions > 64) return fail(NEBEM_EINVAL, "server_create: 1..64 sessions");
    nebem_server_options o;
    if (opt)
        o = *opt;
    else
        nebem_server_default_options(&o);
    if (o.hbm_budget < 4096 || !(o.batch_interactions > 0) || o.max_items < 1 || o.max_items > (1 << 20) ||
        !(o.large_interactions > 0) || o.max_large < 0)
        return fail(NEBEM_EINVAL, "server_create: bad options");
    for (int k = 0; k < nsessions; ++k)
        if (!sessions[k]) return fail(NEBEM_EINVAL, "server_create: NULL session");
    const int mixed = sessions[0]->opt.precision == NEBEM_MIXED;
    for (int k = 0; k < nsessions; ++k)
        if ((sessions[k]->opt.precision == NEBEM_MIXED) != (bool)mixed ||
            sessions[k]->opt.near_factor != sessions[0]->opt.near_factor)
            return fail(NEBEM_EINVAL, "server_create: sessions must share precision and near_factor");
    nebem_server *s = new (std::nothrow) nebem_server;
    if (!s) return fail(NEBEM_ENOMEM, "server_create: host allocation failed");
    s->opt = o;
    s->mixed = mixed;
    s->near_factor = sessions[0]->opt.near_factor;
    for (int k = 0; k < nsessions; ++k) {
        s->geoms.push_back(sessions[k]);
        s->geom_n.push_back(sessions[k]->n);
        // the segments every evaluation path uses, so that served results equal
        // a session evaluation's bit for bit
        const SegPlan sp = seg_plan(sessions[k]->n, sessions[k]->img);
        s->geom_segsz.push_back(sp.segsz);
        s->geom_nseg.push_back(sp.nseg);
    }
    auto bail = [&](hipError_t e, const char *what) {
        nebem_status st = hip_fail(e, what);
        nebem_server_destroy(s);
        return st;
    };
    hipError_t e;
    if ((e = hipGetDevice(&s->device)) != hipSuccess) return bail(e, "hipGetDevice");
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(e, "hipStreamCreate");
    for (int k = 0; k < 2; ++k) {
        if ((e = hipStreamCreateWithFlags(&s->lst[k], hipStreamNonBlocking)) != hipSuccess)
            return bail(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&s->ev_launch[k], hipEventDisableTiming)) != hipSuccess)
            return bail(e, "hipEventCreate");
    }
    if ((e = hipEventCreateWithFlags(&s->ev_adm, hipEventDisableTiming)) != hipSuccess)
        return bail(e, "hipEventCreate");
    if ((e = hipMalloc(&s->arena_dev, (size_t)o.hbm_budget)) != hipSuccess) return bail(e, "hipMalloc(arena)");
    s->arena.init((size_t)o.hbm_budget);
    std::vector<ImgArgs> imgs(nsessions);
    for (int k = 0; k < nsessions; ++k) imgs[k] = sessions[k]->img;
    if ((e = hipMalloc((void **)&s->imgs_dev, sizeof(ImgArgs) * nsessions)) != hipSuccess)
        return bail(e, "hipMalloc(images)");
    if ((e = hipMemcpy(s->imgs_dev, imgs.data(), sizeof(ImgArgs) * nsessions, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(images)");
    s->items_cap = o.max_items;
    s->round_items = eval_items_slots(mixed);
    if (s->round_items < 1 || s->round_items > s->items_cap) s->round_items = 1;
    if ((e = hipMalloc((void **)&s->items_dev, 2 * sizeof(WorkItem) * s->items_cap)) != hipSuccess)
        return bail(e, "hipMalloc(work list)");
    if ((e = hipHostMalloc((void **)&s->items_host, 2 * sizeof(WorkItem) * s->items_cap, hipHostMallocDefault)) !=
        hipSuccess)
        return bail(e, "hipHostMalloc(work list)");
    s->worker = std::thread(worker_main, s);
    *out = s;
    return NEBEM_OK;
}

nebem_status nebem_server_submit(nebem_server *s, int32_t geometry, const double *px, const double *py,
                                 const double *pz, int64_t m, double *phi, double *ex, double *ey, double *ez,
                                 int64_t *ticket)
{
    if (!s || !ticket) return fail(NEBEM_EINVAL, "server_submit: NULL argument");
    if (geometry < 0 || geometry >= (int)s->geoms.size()) return fail(NEBEM_EINVAL, "server_submit: bad geometry");
    if (m < 1 || m > (int64_t)INT32_MAX) return fail(NEBEM_EINVAL, "server_submit: m out of range");
    if (!px || !py || !pz) return fail(NEBEM_EINVAL, "server_submit: NULL point array");
    Request *r = new (std::nothrow) Request;
    if (!r) return fail(NEBEM_ENOMEM, "server_submit: host allocation failed");
    r->geom = geometry;
    r->m = m;
    r->hx = px;
    r->hy = py;
    r->hz = pz;
    r->hphi = phi;
    r->hex = ex;
    r->hey = ey;
    r->hez = ez;
    r->nseg = s->geom_nseg[geometry];
    r->nitems = ((m + 63) / 64) * r->nseg;
    r->ordered = eval_ordering_pays(m);
    r->large = (double)m * (double)s->geom_n[geometry] * s->geoms[geometry]->img_count >= s->opt.large_interactions;
    r->bytes = (size_t)m * (8 + 4 * (size_t)r->nseg) * sizeof(double);
    if (arena_bytes(r->bytes) > s->arena.size) {
        delete r;
        return fail(NEBEM_EBUSY, "server_submit: request larger than the server's HBM budget");
    }
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return fail(NEBEM_EBUSY, "server_submit: server is shutting down");
        }
        r->id = s->next_id++;
        s->all[r->id] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->id;
    return NEBEM_OK;
}

nebem_status nebem_server_wait(nebem_server *s, int64_t ticket, nebem_request_stats *st)
{
    if (!s) return fail(NEBEM_EINVAL, "server_wait: NULL server");
    Request *r = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(NEBEM_EINVAL, "server_wait: unknown ticket");
    r = it->second;
    if (r->waited) return fail(NEBEM_EINVAL, "server_wait: ticket already being waited for");
    r->waited = true;
    s->cv_done.wait(lk, [&] { return r->finished; });
    if (st) {
        st->t_submit = r->t_submit;
        st->t_admit = r->t_admit;
        st->t_done = r->t_done;
        st->points = r->m;
    }
    const nebem_status code = r->status;
    s->all.erase(it);
    delete r;
    if (code) return fail(code, "server_wait: request failed: " + s->worker_error);
    return NEBEM_OK;
}

nebem_status nebem_server_stats(nebem_server *s, nebem_server_counters *out)
{
    if (!s || !out) return fail(NEBEM_EINVAL, "server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->launches = s->launches;
    out->points_done = s->points_done;
    out->interactions = s->interactions_done;
    out->busy_s = s->busy_s;
    out->backfilled = s->adm.backfilled;
    out->queued = (int64_t)s->queue.size();
    out->active = (int64_t)s->active.size();
    return NEBEM_OK;
}

void nebem_server_destroy(nebem_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->all) delete kv.second;
    if (s->items_host) (void)hipHostFree(s->items_host);
    if (s->items_dev) (void)hipFree(s->items_dev);
    if (s->sort_ws) (void)hipFree(s->sort_ws);
    if (s->imgs_dev) (void)hipFree(s->imgs_dev);
    if (s->arena_dev) (void)hipFree(s->arena_dev);
    for (int k = 0; k < 2; ++k) {
        if (s->ev_launch[k]) (void)hipEventDestroy(s->ev_launch[k]);
        if (s->lst[k]) (void)hipStreamDestroy(s->lst[k]);
    }
    if (s->ev_adm) (void)hipEventDestroy(s->ev_adm);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
