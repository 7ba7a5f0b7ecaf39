"""Benchmark: element-point interactions per second on one MI355X.

Workload (default): the single-GEM unit cell -- 8064 rectangular and
right-triangular elements, 121 lattice copies (+-5 along both cell vectors),
1 000 000 evaluation points in the drift and transfer gaps -- in FP64.
One step is the whole hot path on that input: influence-matrix assembly,
LU factorisation and solve, then potential and field at all points.

value = (assembly + evaluation interactions per step) / step time, where an
interaction is one (observation point, element copy) pair.

Prints one JSON line.  Extra keys: per-stage times, the evaluation kernel's
roofline (FP64 vector ALU bound), and the CPU oracle timed on this host's
cores on a bounded sample of the same evaluation.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 floating-point operations per interaction of the evaluation kernel on
# this workload, from rocprofv3 counters (64 x (ADD + MUL + TRANS + 2 FMA)
# FP64 instructions of one evaluation launch / its interactions); see the
# profile summaries committed under profiles/.
FLOPS_PER_INTERACTION = 614.0
# HBM bytes per evaluation launch at the default workload (FETCH_SIZE x 2 +
# WRITE_SIZE x 1, the factors that make a plain 1 GiB copy read 1 GiB and
# write 1 GiB); None when not measured for the current kernel.
EVAL_TRAFFIC_BYTES = 6.912e7
FP64_VALU_PEAK = 78.6e12      # MI355X, FLOP/s
HBM_PEAK = 8.0e12             # B/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--points", type=int, default=1_000_000)
    p.add_argument("--cpu-sample", type=int, default=192, help="points in the oracle's timed sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
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


def cpu_baseline(geom, pts, sigma, n_sample):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    sample = pts[:n_sample]
    t0 = time.perf_counter()
    oracle.eval_points(geom, sigma, sample, nthreads=threads)
    dt = time.perf_counter() - t0
    inter = n_sample * geom.n * geom.images.count
    return {"value": inter / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"evaluation at the first {n_sample} of the benchmark's points "
                      f"({inter:.3e} interactions, {dt:.1f} s)"}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding is not built "
                                   "(--gpus must be 1)"}))
        sys.exit(2)
    import torch

    import paper_2606_24154_amd as nb
    from synth import gem_cell, gem_eval_points

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    geom = gem_cell()
    n, C = geom.n, geom.images.count
    M = args.points
    pts = gem_eval_points(geom, M, seed=1)
    dp = nb.DevicePanels.from_geometry(geom, dev)
    px, py, pz = (torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3))
    b = torch.from_numpy(geom.rhs()).to(dev)
    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    sigma = torch.empty(n, dtype=torch.float64, device=dev)
    out = tuple(torch.empty(M, dtype=torch.float64, device=dev) for _ in range(4))
    stream = torch.cuda.current_stream()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    stage = {"assemble": [], "solve": [], "eval": []}

    prec = nb.MIXED if args.precision == "mixed" else nb.FP64
    info = {}

    def step():
        ev[0].record(stream)
        nb.assemble(dp, A=A, precision=prec)
        ev[1].record(stream)
        _, _, si = nb.solve(A, b, sigma=sigma, ipiv=ipiv, precision=prec)
        info["ir_iters"], info["rel_resid"] = si.ir_iters, si.rel_resid
        ev[2].record(stream)
        nb.eval_points(dp, sigma, px, py, pz, out=out, precision=prec)
        ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()
        stage["assemble"].append(ev[0].elapsed_time(ev[1]))
        stage["solve"].append(ev[1].elapsed_time(ev[2]))
        stage["eval"].append(ev[2].elapsed_time(ev[3]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    inter_asm = n * n * C
    inter_eval = M * n * C
    value = (inter_asm + inter_eval) / (dt / args.steps)
    ms = {k: float(np.mean(v)) for k, v in stage.items()}
    eval_rate = inter_eval / (ms["eval"] * 1e-3)

    roof = None
    if FLOPS_PER_INTERACTION is not None and prec == nb.FP64:
        ach = FLOPS_PER_INTERACTION * inter_eval / (ms["eval"] * 1e-3)
        roof = {"bound": "alu", "kernel": "k_eval_fp64", "achieved": ach / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK,
                "traffic": EVAL_TRAFFIC_BYTES if M == 1_000_000 else None,
                "flops_per_interaction": FLOPS_PER_INTERACTION}

    cpu = None
    if not args.no_cpu:
        # timing only: a seeded density, not the GPU's solution
        s_host = np.random.default_rng(7).normal(0.0, 1e-5, n)
        cpu = cpu_baseline(geom, pts, s_host, args.cpu_sample)

    rec = {
        "metric": "elem-point interactions/s (FP64 vs mixed @1e-6 rel); p50/p99 serve latency",
        "value": value, "unit": "interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == nb.FP64 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"gem_cell: N={n} elements, C={C} copies, M={M} points; "
                               f"assemble + LU solve + evaluate, {args.precision}",
                   "elements": n, "copies": C, "points": M},
        "stages_ms": ms, "eval_interactions_per_s": eval_rate, "solve_info": info,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
