"""Benchmark: element-point interactions per second on one MI355X.

Workload (default): the staggered double thick GEM -- 41 600 rectangular and
right-triangular elements, 121 lattice copies (+-5 along both cell vectors),
4 000 000 evaluation points between the anode and the drift plane -- in
FP64.  The job is the whole hot path on that input: influence-matrix
assembly, LU factorisation and solve with FP64 refinement, then potential
and field at all points.  It is cut into --steps steps: step k evaluates
the k-th slice of the points, step 0 also assembles and solves, so the
timed region holds the job exactly once.

value = (assembly + evaluation interactions of the job) / timed seconds,
where an interaction is one (observation point, element copy) pair.

Prints one JSON line.  Extra keys: per-stage times, the evaluation kernel's
roofline (FP64 vector ALU bound, against the closed forms' algorithmic
operation count), the CPU oracle timed on this host's cores on a bounded
sample of the same evaluation, the mixed-precision job on the same input
(rate, speedup, largest relative difference from the FP64 results), and a
bounded serving replay (continuous batching over resident sessions of the
plates, the GEM cell and this workload, Poisson arrivals) with p50/p99
request latency.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOP per interaction of the closed forms (a transcendental or a
# division counted as one operation): rectangle ~110 arithmetic + 4 sqrt +
# 4 log + 2 atan + 4 div; right triangle ~90 + 3 + 3 + 1 + 3.
ALG_FLOPS_RECT = 124.0
ALG_FLOPS_TRI = 100.0
# Counter figures of the FP64 evaluation kernel per workload, from the
# rocprofv3 runs summarised under profiles/ (FP64 FLOP per interaction =
# 64 x (ADD + MUL + TRANS + 2 FMA) FP64 instructions / interactions; HBM
# bytes per launch = FETCH_SIZE x 2 + WRITE_SIZE, the factors that make a
# plain 1 GiB copy read 1 GiB and write 1 GiB), valid for launches of
# points_per_launch points and only while the evaluation kernel's sources
# hash to source_sha16 (otherwise the counter figures are not reported).
COUNTER_CALIBRATION = {
    # profiles/eval_fp64_thgem_200k.md: one 2e5-point launch, 1.00672e12 interactions
    "thgem": {"flops_per_interaction": 101.04, "valu_per_interaction": 73.09, "traffic_bytes": 537282944,
              "points_per_launch": 200000, "source_sha16": "1b886789b31f0e81"},
}
EVAL_SOURCES = ("field_kernels.hip", "panel_fp64.hpp", "fastmath_fp64.hpp", "poly_coeffs.hpp", "farfield_mixed.hpp",
                "order_kernels.hip", "nebem_internal.hpp")


def _code_only(text):
    """C++ source without comments and with runs of whitespace collapsed
    (the sources hold no comment markers inside string literals)"""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def eval_source_sha16():
    """sha256 (first 16 hex digits) of the evaluation kernel's sources,
    comments and layout left out (so a comment edit does not retire the
    counter figures)"""
    import hashlib
    h = hashlib.sha256()
    for name in EVAL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_24154_amd", "csrc", name)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]
# The paper's own figures, on its own hardware and THGEM model, reported
# beside the measurement as context (they are wall-clock stage times and
# speed-ups, not interaction rates, so no ratio to this benchmark's value
# is formed).
PAPER_CONTEXT = {
    "hardware": "Intel Xeon Gold 6142 (OpenMP, up to 16 threads), 64 GB; NVIDIA T1000 8 GB, "
                "896 CUDA cores at 1395 MHz (Sec. 5.1)",
    "model": "single-layer staggered THGEM, 10 330 elements, 70 periodic repetitions (Sec. 5.2, 5.3)",
    "assembly_min": {"1_thread": 182, "16_threads": 12},
    "inversion": {"cpu_1_thread_min": 63, "cpu_8_threads_min": 14, "gpu_cusolver_s": 31,
                  "gpu_vs_best_cpu": 28},
    "total_solve_min": {"cpu_1_thread": 244.53, "cpu_16_threads": 31.25, "hybrid_16_threads_gpu": 12.49,
                        "speedup_vs_serial": 19.58, "source": "Table 1"},
    "field_map_s": {"points": 2300, "direct": 140.20, "prim_after_5": 47.33, "prim_after_1": 19.12,
                    "source": "Table 2"},
    "fastvolume": "the same map interpolated to within 0.25 % of direct evaluation (Sec. 5.3)",
}
FP64_VALU_PEAK = 78.6e12      # MI355X, FLOP/s
HBM_PEAK = 8.0e12             # B/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", choices=["gem", "thgem", "plates"], default="thgem",
                   help="thgem: staggered double THGEM, 41 600 elements, 4*10^6 points (default, the headline "
                        "figure); gem: single-GEM cell, 8064 elements, 10^6 points; plates: 512-element "
                        "parallel plates")
    p.add_argument("--points", type=int, default=None, help="evaluation points (default per workload)")
    p.add_argument("--cpu-sample", type=int, default=48,
                   help="points in the oracle's timed sample on all host threads (at most 16)")
    p.add_argument("--cpu-sample-1t", type=int, default=3, help="points in the oracle's one-thread timed sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    p.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison step")
    p.add_argument("--serve-requests", type=int, default=120, help="requests in the serving replay (0: skip)")
    p.add_argument("--serve-load", type=float, default=0.8, help="arrival rate / estimated saturation rate")
    p.add_argument("--spacecharge", type=int, default=0, metavar="K",
                   help="instead of the default step: K steps of the dynamic space-charge loop on the GEM "
                        "cell with 10^6 charges (first step re-solves)")
    p.add_argument("--charges", type=int, default=1_000_000)
    p.add_argument("--sc-voxel-um", type=float, default=0.0, metavar="H",
                   help="with --spacecharge: charges reduced to line charges on H um voxels over +-100 um "
                        "(Algorithm 3) in place of the all-pairs sum")
    p.add_argument("--sc-placement", choices=["centre", "weighted"], default="centre",
                   help="with --sc-voxel-um: line placement in each voxel")
    p.add_argument("--serve-matrix", type=int, default=0, metavar="R",
                   help="serving study instead of the step: R requests over the plates, GEM and double-THGEM "
                        "geometries, FP64 saturation measured first, then loads 0.5/0.8/0.95 in FP64 and mixed")
    p.add_argument("--serve-warmup", type=int, default=50, help="serving study: warm-up requests per run")
    p.add_argument("--serve-modes", default="fp64,mixed", help="serving study: precisions, comma-separated")
    p.add_argument("--serve-loads", default="0.5,0.8,0.95", help="serving study: loads to run (of 0.5, 0.8, 0.95)")
    p.add_argument("--serve-batch", type=float, default=None,
                   help="serving study: interactions per server launch (default: the library's)")
    p.add_argument("--serve-max-large", type=int, default=None,
                   help="serving study: large requests (1e11 interactions or more) active at once, 0: no limit "
                        "(default: the library's, one)")
    p.add_argument("--serve-sat", type=float, default=None,
                   help="serving study: FP64 saturation rate (interactions/s) instead of measuring it")
    p.add_argument("--weighting", action="store_true",
                   help="weighting fields of the GEM cell's electrodes (one column per electrode potential "
                        "group) at the evaluation points: one several-column evaluation against one "
                        "evaluation per column")
    p.add_argument("--fastvol", action="store_true",
                   help="FastVolume on the GEM cell's drift gap: grid build (one evaluation at the nodes), "
                        "trilinear lookups at the evaluation points, error against direct evaluation")
    p.add_argument("--adaptive", action="store_true",
                   help="Adaptive Modelling on a periodic strip cell: time and error against the exact sum "
                        "for PrimAfter -1, 5, 3, 2, 1, 0")
    p.add_argument("--voxel", action="store_true",
                   help="point-to-line charge reduction (Algorithm 3) of the space-charge cloud: lines, "
                        "field time at the charges, error against the point-charge field at sample points")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    return p.parse_args()


def copy_probe():
    """A plain copy of known size: 1 GiB read + 1 GiB written.  rocprofv3's
    FETCH_SIZE / WRITE_SIZE for this dispatch calibrate the traffic figures."""
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": x.numel() * 8, "copy_probe_bytes_written": y.numel() * 8}))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(geom, pts, sigma, n_sample, n_sample_1t):
    """The oracle's evaluation timed on this host: on up to 16 threads (the
    host share of one GPU) over the first n_sample points, and on one thread
    over the next n_sample_1t points."""
    import oracle
    threads = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1))
    per_pt = geom.n * geom.images.count
    t0 = time.perf_counter()
    oracle.eval_points(geom, sigma, pts[:n_sample], nthreads=threads)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.eval_points(geom, sigma, pts[n_sample:n_sample + n_sample_1t], nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n_sample * per_pt / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"evaluation at the first {n_sample} of the benchmark's points ({n_sample * per_pt:.3e} "
                      f"interactions, {dt:.1f} s on {threads} threads); one thread: the next {n_sample_1t} "
                      f"points ({n_sample_1t * per_pt:.3e} interactions, {dt1:.1f} s)",
            "value_1_thread": n_sample_1t * per_pt / dt1, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "cpu_model": _cpu_model()}


K_E = 1.0 / (4.0 * math.pi * 8.8541878128e-12)  # Coulomb constant, SI


def point_charge_field(xyz, q, idx, chunk=8):
    """E [len(idx), 3] of the point charges (xyz [n, 3], q [n]) at the
    charges idx, each skipping itself and any charge at its position: the
    exact FP64 sum on the host (numpy), the reference of the line-charge
    accuracy figures."""
    idx = np.asarray(idx)
    E = np.zeros((idx.shape[0], 3))
    for c0 in range(0, idx.shape[0], chunk):
        d = xyz[idx[c0:c0 + chunk]][:, None, :] - xyz[None, :, :]
        r2 = np.einsum("cnk,cnk->cn", d, d)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(r2 > 0.0, q[None, :] / (r2 * np.sqrt(r2)), 0.0)
        E[c0:c0 + chunk] = K_E * np.einsum("cn,cnk->ck", w, d)
    return E


def rel_diff(a, b, floor=1e-3):
    """max pointwise relative difference of phi and |E| (points where the
    reference magnitude is >= floor of its maximum)"""
    ap = np.abs(b[0])
    sel = ap >= floor * ap.max()
    ephi = float(np.max(np.abs(a[0][sel] - b[0][sel]) / ap[sel]))
    en = np.sqrt(b[1] ** 2 + b[2] ** 2 + b[3] ** 2)
    dn = np.sqrt((a[1] - b[1]) ** 2 + (a[2] - b[2]) ** 2 + (a[3] - b[3]) ** 2)
    sel = en >= floor * en.max()
    return ephi, float(np.max(dn[sel] / en[sel]))


def serve_replay(nb, geoms, sessions, n_req, load, eval_rate, seed=4):
    """Config-4 style replay over resident sessions: Poisson arrivals at
    `load` x the saturation rate estimated from the measured evaluation rate,
    geometry uniform, sizes log-uniform in [64, 262144], seeded points."""
    from paper_2606_24154_amd.serving import replay
    from synth import serve_requests, uniform_points
    per_pt = np.mean([g.n * g.images.count for g in geoms])
    mean_pts = (262144 - 64) / np.log(262144 / 64)
    mu_req = eval_rate / (per_pt * mean_pts)
    reqs = serve_requests(n_req, rate_hz=load * mu_req, n_geometries=len(geoms), seed=seed)
    srv = nb.Server(sessions)

    def make_points(g, n, sd):
        return uniform_points(geoms[g].box_lo, geoms[g].box_hi, n, sd)

    run = replay(srv, reqs, make_points)
    c = srv.counters()
    srv.close()
    return {"requests": n_req, "arrival_rate_hz": load * mu_req, "load": load,
            "p50_ms": 1e3 * run["p50_s"], "p99_ms": 1e3 * run["p99_s"],
            "points_per_s": run["points_per_s"], "interactions_per_s": c.interactions / run["span_s"],
            "launches": int(c.launches), "backfilled": int(c.backfilled), "errors": len(run["errors"])}


def serve_matrix(args):
    """Serving over three resident geometries (plates, GEM cell, double
    THGEM), geometry uniform, sizes log-uniform in [64, 262144]: the FP64
    saturation rate is measured by submitting every request at once (or
    taken from --serve-sat); then Poisson arrivals at 0.5 / 0.8 / 0.95 of it
    (the same absolute rates for both precisions, seed 4 + the rate's
    index), each run --serve-warmup requests followed by R measured ones
    (latency statistics over the measured requests only).  Prints one JSON
    line."""
    import torch

    import paper_2606_24154_amd as nb
    from paper_2606_24154_amd.serving import replay
    from synth import gem_cell, parallel_plates, serve_requests, thgem_double, uniform_points

    dev = torch.device("cuda:0")
    geoms = [parallel_plates(), gem_cell(), thgem_double()]
    n_req = args.serve_matrix
    n_warm = args.serve_warmup
    modes = [m for m in args.serve_modes.split(",") if m]
    loads = [float(x) for x in args.serve_loads.split(",") if x]

    def make_points(g, n, sd):
        return uniform_points(geoms[g].box_lo, geoms[g].box_hi, n, sd)

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    def progress(k, n):
        if k % 50 == 0 or k == n:
            log(f"  {k}/{n} requests done")

    def stats(run, reqs, skip):
        lat = run["latency_s"][skip:]
        geo = np.array([g for (_, g, _, _) in reqs[skip:]])
        pct = lambda a, f: 1e3 * float(np.percentile(a, f)) if a.size else None
        return {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": 1e3 * float(lat.max()),
                "mean_ms": 1e3 * float(lat.mean()), "measured": int(lat.size),
                "per_geometry": {geoms[k].name: {"requests": int((geo == k).sum()), "p50_ms": pct(lat[geo == k], 50),
                                                 "p99_ms": pct(lat[geo == k], 99)} for k in range(len(geoms))}}

    out = {"requests": n_req, "warmup_requests": n_warm, "geometries": [g.name for g in geoms],
           "batch_interactions": args.serve_batch or nb.server_default_options().batch_interactions,
           "max_large": (args.serve_max_large if args.serve_max_large is not None
                         else nb.server_default_options().max_large)}
    sat = args.serve_sat
    for name in modes:
        pr = nb.FP64 if name == "fp64" else nb.MIXED
        t0 = time.perf_counter()
        ses = [nb.Session(nb.DevicePanels.from_geometry(g, dev), precision=pr) for g in geoms]
        log(f"{name}: sessions ready in {time.perf_counter() - t0:.1f} s")
        res = {}
        if sat is None:
            burst = [(0.0, g, n, sd) for (_, g, n, sd) in serve_requests(n_req, 1.0, 3, seed=4)]
            work = sum(n * geoms[g].n * geoms[g].images.count for (_, g, n, _) in burst)
            srv = nb.Server(ses, batch_interactions=args.serve_batch, max_large=args.serve_max_large)
            run = replay(srv, burst, make_points, progress)
            srv.close()
            sat = work / run["span_s"]
            out["saturation_interactions_per_s"] = sat
            out["saturation_requests_per_s"] = n_req / run["span_s"]
            out["mean_interactions_per_request"] = work / n_req
            log(f"{name} saturation: {sat:.3e} interactions/s over {run['span_s']:.1f} s")
        else:
            burst = serve_requests(n_req, 1.0, 3, seed=4)
            work = sum(n * geoms[g].n * geoms[g].images.count for (_, g, n, _) in burst)
            out["saturation_interactions_per_s"] = sat
            out["saturation_requests_per_s"] = sat / (work / n_req)
            out["mean_interactions_per_request"] = work / n_req
        for ri, load in enumerate((0.5, 0.8, 0.95)):
            if load not in loads:
                continue
            rate = load * out["saturation_requests_per_s"]
            reqs = serve_requests(n_warm + n_req, rate, 3, seed=4 + ri)
            srv = nb.Server(ses, batch_interactions=args.serve_batch, max_large=args.serve_max_large)
            run = replay(srv, reqs, make_points, progress)
            c = srv.counters()
            srv.close()
            st = stats(run, reqs, n_warm)
            res[str(load)] = {"arrival_rate_hz": rate, **st, "points_per_s": run["points_per_s"],
                              "interactions_per_s": c.interactions / run["span_s"], "launches": int(c.launches),
                              "backfilled": int(c.backfilled), "errors": len(run["errors"])}
            log(f"{name} load {load}: p50 {st['p50_ms']:.0f} ms, p99 {st['p99_ms']:.0f} ms ({st['measured']} requests)")
            # each (precision, load) row as soon as it is measured
            print(json.dumps({"serve_matrix_row": {"precision": name, "load": load, **res[str(load)]}}), flush=True)
        for x in ses:
            x.close()
        del ses
        torch.cuda.empty_cache()
        out[name] = res
    print(json.dumps({"serve_matrix": out}), flush=True)


def weighting_bench(args):
    """Weighting fields (one electrode at 1 V, the others at 0) of the GEM
    cell: multi-RHS solve, then phi/E of every column at the points, once
    with nebem_eval_multi and once column by column; prints one JSON line."""
    import torch

    import paper_2606_24154_amd as nb
    from synth import gem_cell, gem_eval_points

    dev = torch.device("cuda:0")
    g = gem_cell()
    m = args.points or 1_000_000
    val, bc = np.asarray(g.value), np.asarray(g.bc)
    groups = np.unique(val[bc == 0])
    B = np.stack([((bc == 0) & (val == v)).astype(float) for v in groups])
    prec = nb.MIXED if args.precision == "mixed" else nb.FP64
    dp = nb.DevicePanels.from_geometry(g, dev)
    At = nb.assemble(dp)
    sigma, _, _ = nb.solve(At, torch.from_numpy(B).to(dev))
    del At
    pts = gem_eval_points(g, m, seed=1)
    pt = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3)]
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    nb.eval_points_multi(dp, sigma[:, :], pt[0][:4096], pt[1][:4096], pt[2][:4096], precision=prec)  # warm-up
    torch.cuda.synchronize()
    ev[0].record(stream)
    multi = nb.eval_points_multi(dp, sigma, *pt, precision=prec)
    ev[1].record(stream)
    singles = []
    for k in range(len(groups)):
        singles.append(nb.eval_points(dp, sigma[k].contiguous(), *pt, precision=prec))
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_multi = ev[0].elapsed_time(ev[1]) * 1e-3
    t_single = ev[1].elapsed_time(ev[2]) * 1e-3
    same = all(torch.equal(multi[c][k], singles[k][c]) for k in range(len(groups)) for c in range(4))
    K = len(groups)
    inter = float(K) * m * g.n * g.images.count
    print(json.dumps({"metric": "weighting-field evaluation", "unit": "column-interactions/s",
                      "value": inter / t_multi, "higher_is_better": True, "n_gpus": 1, "dtype": args.precision,
                      "config": {"workload": f"gem_cell weighting fields: N={g.n}, C={g.images.count}, M={m}, "
                                             f"{K} electrode columns (potentials {groups.tolist()})"},
                      "columns": K, "ms_multi": 1e3 * t_multi, "ms_column_by_column": 1e3 * t_single,
                      "speedup": t_single / t_multi, "bitwise_equal_to_single_columns": bool(same)}), flush=True)


def fastvol_bench(args):
    """FastVolume (Sec. 3) on the GEM cell's drift gap, from 20 um above the
    top copper to the drift plane, over the centre cell's bounding box:
    a regular 5 um grid, and a graded grid (x, y: uniform 2 um -- the cell's
    box holds parts of the neighbouring holes, so no band of one axis is
    away from every hole; z: 1 um at the foil and at the drift plane,
    growing by 5 % per node up to 10 um in between) --
    each built by one FP64 evaluation at its nodes.  Trilinear lookups at
    10^6 drift-gap points (HIP events); interpolation error against direct
    evaluation at 2*10^4 of them and at 2*10^4 points in the 100 um above
    the grid's foil side, where the hole's field varies fastest."""
    import torch

    import paper_2606_24154_amd as nb
    from synth import gem_cell

    dev = torch.device("cuda:0")
    g = gem_cell()
    ses = nb.Session(nb.DevicePanels.from_geometry(g, dev), precision=nb.FP64)
    sigma = ses.sigma()
    dp = nb.DevicePanels.from_geometry(g, dev)
    z_top = float(g.o[np.asarray(g.value) == -200.0][:, 2].max())
    lo = np.array([0.0, 0.0, z_top + 20e-6])
    hi = np.array([float(g.images.a1[0] + g.images.a2[0]), float(g.images.a2[1]), float(g.box_hi[2]) - 1e-6])
    m = args.points or 1_000_000
    rng = np.random.default_rng(7)
    pts = rng.uniform(lo, hi, (m, 3))
    near = rng.uniform(lo, [hi[0], hi[1], lo[2] + 100e-6], (20000, 3))
    pt = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3)]
    ptn = [torch.from_numpy(np.ascontiguousarray(near[:, k])).to(dev) for k in range(3)]
    ns = min(20000, m)
    direct = np.column_stack([t.cpu().numpy() for t in nb.eval_points(dp, sigma, *(p[:ns] for p in pt))])
    direct_n = np.column_stack([t.cpu().numpy() for t in nb.eval_points(dp, sigma, *ptn)])
    stream = torch.cuda.current_stream()
    q = lambda a: {k: float(np.quantile(a, f)) for k, f in (("p50", 0.5), ("p95", 0.95), ("p99", 0.99),
                                                             ("max", 1.0))}

    def errors(fi, fd, p):
        eE = np.linalg.norm(fi[:, 1:] - fd[:, 1:], axis=1) / np.linalg.norm(fd[:, 1:], axis=1)
        w = int(np.argmax(eE))
        return {"E_rel": q(eE), "frac_E_within_0.25pct": float((eE <= 2.5e-3).mean()),
                "phi_err_over_max_phi": float((np.abs(fi[:, 0] - fd[:, 0]) / np.abs(fd[:, 0]).max()).max()),
                "worst_point_um": [float(1e6 * v) for v in p[w]], "worst_abs_E": float(np.linalg.norm(fd[w, 1:]))}

    def graded_axis(a0, a1, h0, growth, hmax):
        """nodes from a0 to a1 spaced h0 at both ends, growing by `growth`
        per node towards the middle, at most hmax"""
        lo_side, hi_side = [a0], [a1]
        h = h0
        while hi_side[-1] - lo_side[-1] > 2.0 * h:
            lo_side.append(lo_side[-1] + h)
            hi_side.append(hi_side[-1] - h)
            h = min(h * growth, hmax)
        if hi_side[-1] - lo_side[-1] > h:
            lo_side.append(0.5 * (lo_side[-1] + hi_side[-1]))
        return np.array(lo_side + hi_side[::-1])

    h = 5e-6
    shape = tuple(int(np.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))
    step = tuple((hi[a] - lo[a]) / (shape[a] - 1) for a in range(3))
    hxy = 2e-6
    axes = tuple(np.linspace(lo[a], hi[a], int(np.ceil((hi[a] - lo[a]) / hxy)) + 1) for a in range(2)) + \
        (graded_axis(lo[2], hi[2], 1e-6, 1.05, 10e-6),)
    axd = [torch.from_numpy(a).to(dev) for a in axes]
    rows = {}
    for name in ("regular", "graded"):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        if name == "regular":
            vals = nb.fastvol_build(dp, sigma, lo, step, shape)
            look = lambda p: nb.fastvol_interp(vals, lo, step, shape, *p)
            nodes, desc = int(np.prod(shape)), f"{shape[0]}x{shape[1]}x{shape[2]}, step {h * 1e6:.1f} um"
        else:
            vals = nb.fastvol_build_axes(dp, sigma, *axd)
            look = lambda p: nb.fastvol_interp_axes(vals, *axd, *p)
            nodes = int(np.prod([len(a) for a in axes]))
            desc = (f"{len(axes[0])}x{len(axes[1])}x{len(axes[2])}; x, y uniform {hxy * 1e6:.0f} um; z 1 um at "
                    f"the foil and at the drift plane, growing 5 %/node to 10 um in between")
        ev[1].record(stream)
        out = look(pt)  # warm-up
        reps = 20
        torch.cuda.synchronize()
        ev[2].record(stream)
        for _ in range(reps):
            out = look(pt)
        ev[3].record(stream)
        torch.cuda.synchronize()
        t_lookup = ev[2].elapsed_time(ev[3]) * 1e-3 / reps
        fi = np.column_stack([t[:ns].cpu().numpy() for t in out])
        fin = np.column_stack([t.cpu().numpy() for t in look(ptn)])
        rows[name] = {"grid": desc, "nodes": nodes, "build_ms": ev[0].elapsed_time(ev[1]),
                      "lookup_ms": 1e3 * t_lookup, "lookups_per_s": m / t_lookup,
                      "drift_gap": errors(fi, direct, pts[:ns]), "above_foil_100um": errors(fin, direct_n, near)}
        print(f"[fastvol] {name}: {nodes} nodes, lookup {1e3 * t_lookup:.3f} ms, E err max "
              f"{rows[name]['drift_gap']['E_rel']['max']:.2e} (above the foil "
              f"{rows[name]['above_foil_100um']['E_rel']['max']:.2e})", file=sys.stderr, flush=True)
    r = rows["regular"]
    bytes_per_lookup = 24 + 32  # coordinates in, (phi, E) out; the table gathers hit L2 / the die cache
    print(json.dumps({"metric": "FastVolume lookups", "unit": "points/s", "value": r["lookups_per_s"],
                      "higher_is_better": True, "n_gpus": 1, "dtype": "f64",
                      "config": {"workload": f"gem_cell drift gap, M={m} lookups, errors at {ns} drift-gap "
                                             f"points and 20000 points in the 100 um above the foil side"},
                      "roofline": {"bound": "hbm", "achieved": bytes_per_lookup * m / (r["lookup_ms"] * 1e-3) / 1e9,
                                   "peak": 8000.0, "unit": "GB/s",
                                   "frac": bytes_per_lookup * m / (r["lookup_ms"] * 1e-3) / 8e12, "traffic": None},
                      "grids": rows}), flush=True)


def adaptive_bench(args):
    """Adaptive Modelling (Sec. 3 and the paper's PrimAfter table): strip
    cell (4 strips, each 4 primitives along its length, and a mesh plane of
    4 x 4 primitives; every primitive cut into 4 x 16 rectangles; copies
    +-5 x +-5), sigma from the FP64 solve, phi and E at the evaluation
    points for PrimAfter -1 (exact), 5, 3, 2, 1, 0: time and the largest
    error against the exact sum, pointwise relative (points with |x| >=
    1e-3 max|x|) and relative to max|x|."""
    import torch

    import paper_2606_24154_amd as nb
    from synth import strip_cell, uniform_points

    dev = torch.device("cuda:0")
    e, p, emap = strip_cell(sub_u=4, sub_w=16, n_img=5, split=4)
    m = args.points or 200_000
    ses = nb.Session(nb.DevicePanels.from_geometry(e, dev), precision=nb.FP64)
    sigma = ses.sigma()
    dp, dpp = nb.DevicePanels.from_geometry(e, dev), nb.DevicePanels.from_geometry(p, dev)
    demap = torch.from_numpy(emap).to(dev)
    pts = uniform_points(e.box_lo, e.box_hi, m, 11)
    pt = [torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3)]
    nb.eval_points_adaptive(dp, dpp, demap, 0, sigma, pt[0][:4096], pt[1][:4096], pt[2][:4096])  # warm-up
    rows, ref = [], None
    for k in (-1, 5, 3, 2, 1, 0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = nb.eval_points_adaptive(dp, dpp, demap, k, sigma, *pt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        got = np.column_stack([t.cpu().numpy() for t in out])
        if ref is None:
            ref = got
        sel = np.abs(ref[:, 0]) >= 1e-3 * np.abs(ref[:, 0]).max()
        en = np.linalg.norm(ref[:, 1:], axis=1)
        selE = en >= 1e-3 * en.max()
        ephi = float((np.abs(got[sel, 0] - ref[sel, 0]) / np.abs(ref[sel, 0])).max())
        eE = float((np.linalg.norm(got[selE, 1:] - ref[selE, 1:], axis=1) / en[selE]).max())
        nphi = float(np.abs(got[:, 0] - ref[:, 0]).max() / np.abs(ref[:, 0]).max())
        nE = float(np.linalg.norm(got[:, 1:] - ref[:, 1:], axis=1).max() / en.max())
        rows.append({"prim_after": k, "ms": 1e3 * dt, "max_rel_err_phi": ephi, "max_rel_err_E": eE,
                     "max_err_phi_over_max_phi": nphi, "max_err_E_over_max_E": nE})
    print(json.dumps({"metric": "Adaptive Modelling", "unit": "ms", "n_gpus": 1, "dtype": "f64",
                      "config": {"workload": f"strip cell: N={e.n} elements in {p.n} primitives, "
                                             f"C={e.images.count} copies, M={m} points"},
                      "rows": rows}), flush=True)


def voxel_bench(args):
    """Algorithm 3 on an avalanche-like cloud of 10^6 charges: +e ions and
    -e electrons, each a Gaussian of sigma 20 um, their centres 20 um apart
    along z (an interleaved neutral cloud has no coarse structure for lines
    to keep); line charges on 5 and 10 um voxels over +-100 um, both line
    placements.  Per row: the reduction, the lines' field at every charge
    (HIP events), and the error of the charges' own field at 400 sampled
    charges against the exact point-charge sum (FP64, numpy, on the host), for
    the lines alone and for the field with the 27 voxels around each charge
    taken as point charges."""
    import torch

    import paper_2606_24154_amd as nb
    from synth import charge_cloud

    dev = torch.device("cuda:0")
    n = args.charges
    xi, _ = charge_cloud([0.0, 0.0, -10e-6], 20e-6, n // 2, seed=3)
    xe, _ = charge_cloud([0.0, 0.0, 10e-6], 20e-6, n - n // 2, seed=4)
    xyz = np.concatenate([xi, xe])
    q = np.concatenate([np.full(n // 2, 1.602176634e-19), np.full(n - n // 2, -1.602176634e-19)])
    qd = [torch.from_numpy(np.ascontiguousarray(xyz[:, k])).to(dev) for k in range(3)]
    qq = torch.from_numpy(q).to(dev)
    sample = np.random.default_rng(5).choice(n, 400, replace=False)
    ref = point_charge_field(xyz, q, sample)
    refn = np.linalg.norm(ref, axis=1)
    stream = torch.cuda.current_stream()
    stats = lambda e: {"p50": float(np.median(e)), "p90": float(np.quantile(e, 0.9)), "max": float(e.max())}
    rows = []
    for h in (5e-6, 10e-6):
        nv = int(round(200e-6 / h))
        grid = ((-100e-6,) * 3, (h,) * 3, (nv,) * 3)
        for placement in ("centre", "weighted"):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            ev[0].record(stream)
            lines, out = nb.voxelize_charges(*qd, qq, *grid, placement=placement)
            ev[1].record(stream)
            f = nb.line_field(lines, *qd)
            ev[2].record(stream)
            E, nl = nb.charge_field_lines(*qd, qq, *grid, placement=placement)
            ev[3].record(stream)
            torch.cuda.synchronize()
            plain = np.column_stack([t.cpu().numpy() for t in f[1:]])[sample]
            near = np.column_stack([t.cpu().numpy() for t in E])[sample]
            with np.errstate(invalid="ignore"):
                e_plain = np.linalg.norm(plain - ref, axis=1) / refn
            e_near = np.linalg.norm(near - ref, axis=1) / refn
            rows.append({"voxel_um": h * 1e6, "placement": placement, "lines": int(lines.shape[0]),
                         "outside": int(out), "reduce_ms": ev[0].elapsed_time(ev[1]),
                         "lines_field_at_charges_ms": ev[1].elapsed_time(ev[2]),
                         "near_exact_field_at_charges_ms": ev[2].elapsed_time(ev[3]),
                         "segment_interactions_per_s": float(lines.shape[0]) * n / (ev[1].elapsed_time(ev[2]) * 1e-3),
                         "E_rel_err_lines_only": stats(np.nan_to_num(e_plain, nan=np.inf)),
                         "E_rel_err_near_exact": stats(e_near)})
            print(f"[voxel] {h * 1e6:.0f} um {placement}: {rows[-1]['lines']} lines, near-exact field "
                  f"{rows[-1]['near_exact_field_at_charges_ms']:.1f} ms, E err p50 "
                  f"{rows[-1]['E_rel_err_near_exact']['p50']:.2e} (lines only "
                  f"{rows[-1]['E_rel_err_lines_only']['p50']:.2e})", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "point-to-line charge reduction", "unit": "ms", "n_gpus": 1, "dtype": "f64",
                      "config": {"workload": f"{n} charges (+e and -e Gaussians of 20 um, centres 20 um apart), "
                                             f"voxel grids over +-100 um; the charges' own field at 400 sampled "
                                             f"charges against the exact point sum"},
                      "rows": rows}), flush=True)


def spacecharge_bench(args):
    """Config 3: GEM cell, charges ~ N(hole centre, 20 um), +-e alternating;
    each step = (re-solve every 10th step) + panel field at every charge +
    all-pairs charge field (or, with --sc-voxel-um, the field of the
    charges' line charges) + Euler move."""
    import torch

    import paper_2606_24154_amd as nb
    from synth import charge_cloud, gem_cell

    dev = torch.device("cuda:0")
    geom = gem_cell()
    prec = nb.MIXED if args.precision == "mixed" else nb.FP64
    ses = nb.Session(nb.DevicePanels.from_geometry(geom, dev), precision=prec)
    centre = [0.5 * (geom.images.a1[0] + geom.images.a2[0]), 0.5 * geom.images.a2[1], 0.0]
    xyz, q = charge_cloud(centre, 20e-6, args.charges, seed=3)
    qx, qy, qz = (torch.from_numpy(np.ascontiguousarray(xyz[:, k])).to(dev) for k in range(3))
    qd = torch.from_numpy(q).to(dev)
    E = tuple(torch.empty(len(q), dtype=torch.float64, device=dev) for _ in range(3))
    stream = torch.cuda.current_stream()
    # panel-only time at the charges (the same launch the step makes)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    ses.eval_points(qx, qy, qz)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_panel = ev[0].elapsed_time(ev[1]) * 1e-3
    times, nlines = [], []
    h = args.sc_voxel_um * 1e-6
    if h > 0:
        nv = int(round(200e-6 / h))
        vox = ([c - 100e-6 for c in centre], (h,) * 3, (nv,) * 3)
    for k in range(args.spacecharge):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if h > 0:
            nlines.append(ses.spacecharge_step_lines(qx, qy, qz, qd, k, *vox, E=E, placement=args.sc_placement)[1])
        else:
            ses.spacecharge_step(qx, qy, qz, qd, k, E=E)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    nq = len(q)
    t_plain = float(np.median(times[1:])) if len(times) > 1 else times[0]
    pairs = nq * (nq - 1)
    panel_inter = nq * geom.n * geom.images.count
    rec = {"metric": "space-charge step time", "value": 1e3 * t_plain, "unit": "ms/step",
           "higher_is_better": False, "n_gpus": 1, "steps": args.spacecharge, "dtype": args.precision,
           "config": {"workload": f"gem_cell + {nq} point charges (+-e), N={geom.n}, C={geom.images.count}, "
                                  f"dt=1 ps, mobility 1e-4 m^2/Vs, re-solve every 10 steps"
                                  + (f"; charges as line charges on {args.sc_voxel_um} um voxels" if h > 0 else "")},
           "step_ms": [1e3 * t for t in times], "panel_part_ms": 1e3 * t_panel,
           "panel_interactions_per_s": panel_inter / t_panel,
           "resolve_step_ms": 1e3 * times[0]}
    if h > 0:
        rec["lines"] = nlines
    else:
        rec["pair_interactions_per_s"] = pairs / max(t_plain - t_panel, 1e-9)
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.weighting:
        weighting_bench(args)
        return
    if args.fastvol:
        fastvol_bench(args)
        return
    if args.adaptive:
        adaptive_bench(args)
        return
    if args.voxel:
        voxel_bench(args)
        return
    if args.spacecharge:
        spacecharge_bench(args)
        return
    if args.serve_matrix:
        serve_matrix(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding is not built "
                                   "(--gpus must be 1)"}))
        sys.exit(2)
    headline(args)


def headline(args):
    """The default bench line: the whole job of one workload (assembly, LU
    solve with refinement, evaluation at all M points) cut into `steps`
    steps -- step k evaluates the k-th of `steps` equal slices of the points,
    and step 0 also assembles and solves -- so that the timed region holds
    the job exactly once.  value = (N^2 C + M N C) interactions / timed
    seconds.  Warm-up steps run steps 0 .. warmup-1 of the same job."""
    import torch

    import paper_2606_24154_amd as nb
    from synth import gem_cell, gem_eval_points, parallel_plates, thgem_double, thgem_eval_points, uniform_points

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    if args.workload == "gem":
        geom = gem_cell()
        M = args.points or 1_000_000
        pts = gem_eval_points(geom, M, seed=1)
    elif args.workload == "thgem":
        geom = thgem_double()
        M = args.points or 4_000_000
        pts = thgem_eval_points(geom, M, seed=2)
    else:
        geom = parallel_plates()
        M = args.points or 4096
        pts = uniform_points(geom.box_lo, geom.box_hi, M, 0)
    n, C = geom.n, geom.images.count
    K = max(1, args.steps)
    dp = nb.DevicePanels.from_geometry(geom, dev)
    px, py, pz = (torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3))
    b = torch.from_numpy(geom.rhs()).to(dev)
    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    sigma = torch.empty(n, dtype=torch.float64, device=dev)
    out = tuple(torch.empty(M, dtype=torch.float64, device=dev) for _ in range(4))
    bounds = np.linspace(0, M, K + 1).round().astype(np.int64)
    stream = torch.cuda.current_stream()
    prec = nb.MIXED if args.precision == "mixed" else nb.FP64
    info = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
    log(f"{geom.name}: N={n}, C={C}, M={M}, {K} steps; set-up {time.perf_counter() - t_setup:.1f} s")

    def step(k):
        """step k of the job; returns (assemble ms, solve ms, eval ms, points)"""
        i0, i1 = int(bounds[k]), int(bounds[k + 1])
        ev[0].record(stream)
        if k == 0:
            nb.assemble(dp, A=A, precision=prec)
            ev[1].record(stream)
            _, _, si = nb.solve(A, b, sigma=sigma, ipiv=ipiv, precision=prec)
            info["ir_iters"], info["rel_resid"] = si.ir_iters, si.rel_resid
        else:
            ev[1].record(stream)
        ev[2].record(stream)
        if i1 > i0:
            nb.eval_points(dp, sigma, px[i0:i1], py[i0:i1], pz[i0:i1], out=tuple(o[i0:i1] for o in out),
                           precision=prec)
        ev[3].record(stream)
        torch.cuda.synchronize()
        return (ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]), i1 - i0)

    for w in range(args.warmup):
        t = step(w % K)
        log(f"warmup {w}: assemble {t[0]:.1f} ms, solve {t[1]:.1f} ms, eval {t[2]:.1f} ms ({t[3]} points)")
    stages = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        t = step(k)
        stages.append(t)
        log(f"step {k}: assemble {t[0]:.1f} ms, solve {t[1]:.1f} ms, eval {t[2]:.1f} ms ({t[3]} points)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inter_asm = n * n * C
    inter_eval = M * n * C
    value = (inter_asm + inter_eval) / dt
    t_asm, t_solve = stages[0][0], stages[0][1]
    t_eval = sum(t[2] for t in stages)
    eval_rate = inter_eval / (t_eval * 1e-3)

    roof = None
    if prec == nb.FP64:
        # algorithmic FLOP per interaction: the closed forms' operation counts,
        # a transcendental or division counted as one operation, over this
        # geometry's mix of rectangles and right triangles
        kind = np.asarray(geom.kind)
        n_rect, n_tri = int((kind == 0).sum()), int((kind == 1).sum())
        f_alg = (n_rect * ALG_FLOPS_RECT + n_tri * ALG_FLOPS_TRI) / n
        # average over the evaluation launches (one per step; their points
        # differ by at most one), HIP events on the launching stream
        per_launch_ms = t_eval / K
        per_launch_inter = inter_eval / K
        ach = f_alg * per_launch_inter / (per_launch_ms * 1e-3)
        cal = COUNTER_CALIBRATION.get(args.workload)
        sha = eval_source_sha16()
        if cal and cal.get("source_sha16") != sha:
            cal = None  # the kernel changed since the counters were taken
        roof = {"bound": "alu", "kernel": "k_eval_fp64", "achieved": ach / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK,
                "traffic": cal["traffic_bytes"] if (cal and cal["points_per_launch"] == round(M / K)) else None,
                "flops_per_interaction": f_alg, "flops_per_interaction_kind": "algorithmic",
                "elements": {"rectangles": n_rect, "right_triangles": n_tri},
                "launches": K, "avg_launch_ms": per_launch_ms, "interactions_per_launch": per_launch_inter,
                "eval_source_sha16": sha}
        if cal:
            roof["counter_flops_per_interaction"] = cal["flops_per_interaction"]
            roof["counter_frac"] = cal["flops_per_interaction"] * eval_rate / FP64_VALU_PEAK

    mixed = None
    if not args.no_mixed and prec == nb.FP64:
        torch.cuda.synchronize()
        ref = [t.cpu().numpy() for t in out]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        t1 = time.perf_counter()
        e[0].record(stream)
        nb.assemble(dp, A=A, precision=nb.MIXED)
        e[1].record(stream)
        _, _, si = nb.solve(A, b, sigma=sigma, ipiv=ipiv, precision=nb.MIXED)
        e[2].record(stream)
        nb.eval_points(dp, sigma, px, py, pz, out=out, precision=nb.MIXED)
        e[3].record(stream)
        torch.cuda.synchronize()
        dt_m = time.perf_counter() - t1
        got = [t.cpu().numpy() for t in out]
        ephi, eE = rel_diff(got, ref)
        log(f"mixed job: {1e3 * dt_m:.1f} ms (assemble {e[0].elapsed_time(e[1]):.1f}, solve "
            f"{e[1].elapsed_time(e[2]):.1f}, eval {e[2].elapsed_time(e[3]):.1f} ms)")
        mixed = {"value": (inter_asm + inter_eval) / dt_m, "job_ms": 1e3 * dt_m,
                 "stages_ms": {"assemble": e[0].elapsed_time(e[1]), "solve": e[1].elapsed_time(e[2]),
                               "eval": e[2].elapsed_time(e[3])},
                 "eval_interactions_per_s": inter_eval / (e[2].elapsed_time(e[3]) * 1e-3),
                 "speedup_vs_fp64": dt / dt_m, "ir_iters": si.ir_iters,
                 "rel_resid": si.rel_resid, "max_rel_diff_vs_fp64": {"phi": ephi, "E": eE}}
    del A
    torch.cuda.empty_cache()

    serve = None
    if args.serve_requests > 0 and prec == nb.FP64:
        geoms = [parallel_plates(), gem_cell(), geom] if args.workload == "thgem" else [parallel_plates(), geom]
        serve = {}
        for name, pr in (("fp64", nb.FP64), ("mixed", nb.MIXED)):
            t1 = time.perf_counter()
            ses = [nb.Session(nb.DevicePanels.from_geometry(g, dev), precision=pr) for g in geoms]
            log(f"serve {name}: {len(ses)} sessions ready in {time.perf_counter() - t1:.1f} s")
            serve[name] = serve_replay(nb, geoms, ses, args.serve_requests, args.serve_load, eval_rate)
            log(f"serve {name}: p50 {serve[name]['p50_ms']:.0f} ms, p99 {serve[name]['p99_ms']:.0f} ms")
            for x in ses:
                x.close()
            del ses
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        # timing only: a seeded density, not the GPU's solution
        s_host = np.random.default_rng(7).normal(0.0, 1e-5, n)
        cpu = cpu_baseline(geom, pts, s_host, args.cpu_sample, args.cpu_sample_1t)
        log(f"oracle: {cpu['value']:.3e} interactions/s on {cpu['cores']} threads, "
            f"{cpu['value_1_thread']:.3e} on 1")

    rec = {
        "metric": "elem-point interactions/s (FP64 vs mixed @1e-6 rel); p50/p99 serve latency",
        "value": value, "unit": "interactions/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == nb.FP64 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"{geom.name}: N={n} elements, C={C} copies, M={M} points; assemble + LU solve "
                               f"(+ refinement) + evaluate, {args.precision}; the job cut into {K} steps "
                               f"(step k evaluates slice k of the points, step 0 also assembles and solves)",
                   "elements": n, "copies": C, "points": M},
        "job_s": dt, "stages_ms": {"assemble": t_asm, "solve": t_solve, "eval_total": t_eval},
        "eval_interactions_per_s": eval_rate, "solve_info": info,
        "roofline": roof, "cpu_baseline": cpu, "mixed": mixed, "serve": serve,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(rec), flush=True)
    # release device memory before the interpreter tears down
    del out, px, py, pz, b, ipiv, sigma, dp
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
