"""The seeded synthetic inputs keep the shapes the benchmarks and the
evaluation path rely on: element counts and mixes of the three geometries;
well-formed elements (positive legs, perpendicular for rectangles and right
triangles); every right triangle of the GEM cell and the double THGEM in a
consecutive pair (two halves of one triangle: same right-angle corner, one
shared leg, the other legs opposite), the structure the paired evaluation
uses; reproducible points, charge clouds and request streams (same seed,
same values); the serving stream's size law."""
import math

import numpy as np
import pytest

from synth import charge_cloud, gem_cell, parallel_plates, serve_requests, thgem_double, uniform_points
from synth.geometry import CONDUCTOR, DIELECTRIC


def _pairs(g):
    """Indices i where elements i, i + 1 are the two halves of one triangle."""
    kind, o, u, w = np.asarray(g.kind), np.asarray(g.o), np.asarray(g.u), np.asarray(g.w)
    scale = np.abs(o).max()
    eq = lambda a, b: np.abs(a - b).max() <= 1e-12 * scale
    out, i = [], 0
    while i < g.n - 1:
        ok = False
        if kind[i] == 1 and kind[i + 1] == 1 and eq(o[i], o[i + 1]):
            for s1, t1 in ((u[i], w[i]), (w[i], u[i])):
                for s2, t2 in ((u[i + 1], w[i + 1]), (w[i + 1], u[i + 1])):
                    if eq(s1, s2) and np.dot(t1, t2) < 0 and \
                            np.linalg.norm(np.cross(t1, t2)) <= 1e-9 * np.linalg.norm(t1) * np.linalg.norm(t2):
                        ok = True
        if ok:
            out.append(i)
            i += 2
        else:
            i += 1
    return out


@pytest.fixture(scope="module")
def geoms():
    return {"plates": parallel_plates(), "gem": gem_cell(), "thgem": thgem_double()}


def test_counts_and_mix(geoms):
    want = {"plates": (512, 512, 0), "gem": (8064, 128, 7936), "thgem": (41600, 2688, 38912)}
    for name, (n, n_rect, n_tri) in want.items():
        kind = np.asarray(geoms[name].kind)
        assert (geoms[name].n, int((kind == 0).sum()), int((kind == 1).sum())) == (n, n_rect, n_tri), name
    bc = np.asarray(geoms["gem"].bc)
    assert int((bc == DIELECTRIC).sum()) == 1536 and int((bc == CONDUCTOR).sum()) == 8064 - 1536


def test_elements_well_formed(geoms):
    for name, g in geoms.items():
        u, w = np.asarray(g.u), np.asarray(g.w)
        lu, lw = np.linalg.norm(u, axis=1), np.linalg.norm(w, axis=1)
        assert lu.min() > 0 and lw.min() > 0, name
        cos = np.abs(np.einsum("ij,ij->i", u, w)) / (lu * lw)
        assert cos.max() < 1e-9, (name, cos.max())
        assert np.max(np.maximum(lu, lw) / np.minimum(lu, lw)) <= 5.5 + 1e-9 or name == "plates", name


def test_every_triangle_in_a_consecutive_pair(geoms):
    for name in ("gem", "thgem"):
        g = geoms[name]
        n_tri = int((np.asarray(g.kind) == 1).sum())
        assert 2 * len(_pairs(g)) == n_tri, name


def test_seeded_inputs_reproducible():
    lo, hi = np.zeros(3), np.ones(3)
    a, b = uniform_points(lo, hi, 1000, 5), uniform_points(lo, hi, 1000, 5)
    assert np.array_equal(a, b) and not np.array_equal(a, uniform_points(lo, hi, 1000, 6))
    assert a.min() >= 0 and a.max() < 1
    x1, q1 = charge_cloud((0, 0, 0), 20e-6, 1000, seed=3)
    x2, q2 = charge_cloud((0, 0, 0), 20e-6, 1000, seed=3)
    assert np.array_equal(x1, x2) and np.array_equal(q1, q2) and q1.sum() == 0
    assert serve_requests(50, 5.0, 3, seed=4) == serve_requests(50, 5.0, 3, seed=4)


def test_serve_request_sizes_log_uniform():
    reqs = serve_requests(20000, 10.0, 3, seed=11)
    n = np.array([r[2] for r in reqs])
    assert n.min() >= 64 and n.max() <= 262144
    # log-uniform on [64, 262144]: median at the geometric mean 4096
    assert abs(np.log(np.median(n)) - math.log(4096)) < 0.1
    g = np.array([r[1] for r in reqs])
    assert set(g.tolist()) == {0, 1, 2} and abs(np.mean(g == 0) - 1 / 3) < 0.02
    t = np.array([r[0] for r in reqs])
    assert np.all(np.diff(t) >= 0) and abs(len(t) / t[-1] - 10.0) < 0.3
