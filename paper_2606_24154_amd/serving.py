"""Open-loop load replay for the continuous-batching server: requests arrive
at given times (e.g. Poisson), each naming a resident geometry and a batch
of points; latency is the server's own submit-to-results time.  Host-side
scheduling only -- every evaluation runs in the library's kernels."""
from __future__ import annotations

import threading
import time

import numpy as np


def replay(server, requests, make_points, progress=None):
    """requests: list of (arrival_s, geometry, n_points, seed) sorted by
    arrival; make_points(geometry, n, seed) -> (n, 3) float64.  Returns a dict
    with per-request latencies (s), points/s and the span of the run.
    progress(k, n), if given, is called after each completed request."""
    pts = [make_points(g, n, sd) for (_, g, n, sd) in requests]
    tickets = [None] * len(requests)
    submitted = [threading.Event() for _ in requests]
    errors = []

    def submitter():
        t0 = time.perf_counter()
        for k, (t_arr, g, n, sd) in enumerate(requests):
            dt = t_arr - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            try:
                tickets[k] = server.submit(g, pts[k], want=("phi", "ex", "ey", "ez"))
            except Exception as e:  # recorded, the run continues
                errors.append((k, repr(e)))
            submitted[k].set()

    th = threading.Thread(target=submitter)
    th.start()
    lat, t_first, t_last, npts = [], None, None, 0
    results = [None] * len(requests)
    # collect results in submission order while later requests still arrive
    for k in range(len(requests)):
        submitted[k].wait()
        t = tickets[k]
        if t is None:
            continue
        out, st = server.wait(t)
        results[k] = out
        if progress is not None:
            progress(k + 1, len(requests))
        lat.append(st.t_done - st.t_submit)
        t_first = st.t_submit if t_first is None else min(t_first, st.t_submit)
        t_last = st.t_done if t_last is None else max(t_last, st.t_done)
        npts += int(st.points)
    th.join()
    lat = np.array(lat)
    span = (t_last - t_first) if lat.size else 0.0
    return {
        "latency_s": lat, "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        "points": npts, "span_s": span, "points_per_s": npts / span if span > 0 else None,
        "errors": errors, "results": results, "points_in": pts,
    }
