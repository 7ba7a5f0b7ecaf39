"""Seeded evaluation points, charge clouds and serving request streams.

All random numbers come from numpy's PCG64 (`numpy.random.default_rng`).
Points are drawn as lo + (hi - lo) * U[0,1)^3 in the stated region.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry

E_CHARGE = 1.602176634e-19  # elementary charge, C (SI 2019 exact value)


def uniform_points(lo, hi, m: int, seed: int) -> np.ndarray:
    """m points uniform in the axis-aligned box [lo, hi), f64 [m, 3]."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    return lo + (hi - lo) * rng.random((m, 3))


def _cell_points(rng, a1, a2, m):
    st = rng.random((m, 2))
    return st[:, :1] * a1[None, :2] + st[:, 1:] * a2[None, :2]


def gem_eval_points(geom: Geometry, m: int, seed: int = 1) -> np.ndarray:
    """Uniform in the centre lattice cell; the first half in the drift gap
    (top copper to drift plane), the second half in a 1 mm transfer gap below
    the bottom copper."""
    rng = np.random.default_rng(seed)
    a1, a2 = geom.images.a1, geom.images.a2
    xy = _cell_points(rng, a1, a2, m)
    z_top = float(geom.o[geom.value == -200.0][:, 2].max())
    z_bot = float(geom.o[geom.value == 200.0][:, 2].min())
    z_drift = float(geom.box_hi[2])
    r = rng.random(m)
    h = m // 2
    z = np.empty(m)
    z[:h] = z_top + (z_drift - z_top) * r[:h]
    z[h:] = (z_bot - 1e-3) + 1e-3 * r[h:]
    return np.column_stack([xy, z])


def thgem_eval_points(geom: Geometry, m: int, seed: int = 2) -> np.ndarray:
    """Uniform in the centre lattice cell between anode and drift cathode."""
    rng = np.random.default_rng(seed)
    xy = _cell_points(rng, geom.images.a1, geom.images.a2, m)
    z = geom.box_lo[2] + (geom.box_hi[2] - geom.box_lo[2]) * rng.random(m)
    return np.column_stack([xy, z])


def charge_cloud(center, sigma: float, n: int, seed: int = 3):
    """n point charges ~ N(center, sigma^2 I); alternating +e (ions) and -e
    (electrons), so the cloud is neutral for even n.  Returns (xyz [n,3], q [n])."""
    rng = np.random.default_rng(seed)
    xyz = np.asarray(center, float)[None, :] + sigma * rng.standard_normal((n, 3))
    q = np.where(np.arange(n) % 2 == 0, E_CHARGE, -E_CHARGE).astype(np.float64)
    return xyz, q


def serve_requests(n_requests: int, rate_hz: float, n_geometries: int, seed: int,
                   n_min: int = 64, n_max: int = 262144):
    """Poisson arrivals at `rate_hz`; each request names a geometry uniformly
    and a point count n = floor(exp(U[ln n_min, ln n_max])).  Returns a list of
    (arrival_time_s, geometry_index, n_points, point_seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    g = rng.integers(0, n_geometries, n_requests)
    n = np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_requests))).astype(int)
    n = np.clip(n, n_min, n_max)
    ps = rng.integers(0, 2**31 - 1, n_requests)
    return [(float(t[i]), int(g[i]), int(n[i]), int(ps[i])) for i in range(n_requests)]
