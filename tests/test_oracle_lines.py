"""Pins of the oracle's point-to-line reduction (Algorithm 3) and of the
uniform line-segment field: the segment's potential and field against
adaptive quadrature of point charges along it, the point-charge limit far
away, E = -grad phi, and the voxel reduction's charge conservation and
placement."""
import numpy as np
from scipy import integrate

import oracle

KE = oracle.ke()


def test_segment_against_quadrature():
    rng = np.random.default_rng(0)
    A, B, lam = np.array([1e-6, -2e-6, 3e-6]), np.array([4e-6, 2e-6, 9e-6]), 2.5e-9
    L = np.linalg.norm(B - A)
    pts = A + rng.uniform(-20e-6, 20e-6, (12, 3))
    got = oracle.line_field([[*A, *B, lam]], pts)
    for p, g in zip(pts, got):
        f = lambda s, c: (KE * lam * ((p - (A + s * (B - A) / L))[c - 1] if c else 1.0)
                          / np.linalg.norm(p - (A + s * (B - A) / L)) ** (3 if c else 1))
        ref = [integrate.quad(f, 0, L, args=(c,), epsabs=0, epsrel=1e-13, limit=200)[0] for c in range(4)]
        np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_far_field_is_point_charge_and_gradient():
    A, B, lam = np.array([0.0, 0.0, 0.0]), np.array([0.0, 0.0, 1e-6]), 1e-9
    Q = lam * 1e-6
    p = np.array([[3e-3, -2e-3, 4e-3]])
    r = np.linalg.norm(p[0] - np.array([0, 0, 0.5e-6]))
    got = oracle.line_field([[*A, *B, lam]], p)[0]
    assert abs(got[0] - KE * Q / r) <= 1e-7 * KE * Q / r
    # E = -grad phi by central differences near the segment
    p0 = np.array([2e-6, 1e-6, 0.3e-6])
    h = 1e-10
    grad = [(oracle.line_field([[*A, *B, lam]], [p0 + h * e])[0, 0]
             - oracle.line_field([[*A, *B, lam]], [p0 - h * e])[0, 0]) / (2 * h) for e in np.eye(3)]
    np.testing.assert_allclose(oracle.line_field([[*A, *B, lam]], [p0])[0, 1:], -np.array(grad), rtol=1e-6)


def test_voxel_reduction():
    rng = np.random.default_rng(1)
    xyz = rng.normal(0, 10e-6, (2000, 3))
    q = np.where(np.arange(2000) % 2, 1.0, -1.0) * 1.602176634e-19
    origin, step, shape = (-30e-6, -30e-6, -30e-6), (5e-6, 5e-6, 5e-6), (12, 12, 12)
    lines, out = oracle.voxel_lines(xyz, q, origin, step, shape)
    inside = np.all(np.abs(xyz) < 30e-6, axis=1)
    assert out == (~inside).sum()
    np.testing.assert_allclose((lines[:, 6] * step[2]).sum(), q[inside].sum(), atol=1e-30)
    # every segment lies in its voxel, parallel to z, one voxel tall
    assert np.allclose(lines[:, 5] - lines[:, 2], step[2], rtol=1e-12) and np.all(lines[:, 0] == lines[:, 3])
    ix = np.floor((lines[:, 0] - origin[0]) / step[0])
    assert np.all((ix >= 0) & (ix < shape[0]))
    # a lone charge: by default its line runs through the voxel centre; with
    # the weighted placement through the charge itself
    one, _ = oracle.voxel_lines([[1e-6, 2e-6, 3e-6]], [2.0], origin, step, shape)
    np.testing.assert_allclose(one[0, [0, 1]], [2.5e-6, 2.5e-6], rtol=1e-12)
    assert one[0, 6] == 2.0 / step[2]
    one, _ = oracle.voxel_lines([[1e-6, 2e-6, 3e-6]], [2.0], origin, step, shape, placement="weighted")
    np.testing.assert_array_equal(one[0, [0, 1]], [1e-6, 2e-6])


def _cloud(n, centre, sigma, seed):
    rng = np.random.default_rng(seed)
    xyz = np.asarray(centre) + rng.normal(0, sigma, (n, 3))
    q = np.where(np.arange(n) % 2, 1.0, -1.0) * 1.602176634e-19 * rng.uniform(0.5, 2.0, n)
    return xyz, q


def test_charge_field_lines_all_near_is_the_point_sum():
    """On a 2 x 2 x 2 grid every voxel is a neighbour of every other, so no
    line is used: the field is the plain sum over the other charges."""
    xyz, q = _cloud(300, [0, 0, 0], 4e-6, 2)
    origin, step, shape = (-20e-6,) * 3, (20e-6,) * 3, (2, 2, 2)
    assert np.all(np.abs(xyz) < 20e-6)
    E, S = oracle.charge_field_lines(xyz, q, origin, step, shape)
    ref = oracle.coulomb(xyz, xyz, q, np.arange(len(q)))[:, 1:]
    np.testing.assert_allclose(E, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.all(S >= np.linalg.norm(ref, axis=1) * (1 - 1e-12))


def test_charge_field_lines_far_cluster_as_lines():
    """Two clusters, each within two neighbouring voxels and five voxels
    from the other: a charge of one feels its own cluster charge by charge
    and the other cluster through that cluster's lines only; a charge
    outside the grid feels every line."""
    a, qa = _cloud(200, [-15e-6, 2.5e-6, 2.5e-6], 0.6e-6, 3)
    b, qb = _cloud(200, [20e-6, 2.5e-6, 2.5e-6], 0.6e-6, 4)
    origin, step, shape = (-25e-6, -5e-6, -5e-6), (5e-6, 5e-6, 5e-6), (10, 2, 2)
    xyz, q = np.vstack([a, b]), np.concatenate([qa, qb])
    # cluster a within x voxels 1..2, cluster b within 8..9
    ia = np.floor((a[:, 0] - origin[0]) / step[0])
    ib = np.floor((b[:, 0] - origin[0]) / step[0])
    assert ia.min() >= 1 and ia.max() <= 2 and ib.min() >= 8 and ib.max() <= 9
    assert np.all(np.abs(xyz[:, 1:] - 2.5e-6) < 7.5e-6)
    for placement in ("centre", "weighted"):
        E, _ = oracle.charge_field_lines(xyz, q, origin, step, shape, placement)
        lb, _ = oracle.voxel_lines(b, qb, origin, step, shape, placement)
        ref = oracle.coulomb(a, a, qa, np.arange(len(qa)))[:, 1:] + oracle.line_field(lb, a)[:, 1:]
        np.testing.assert_allclose(E[:len(a)], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    # a charge outside the grid
    out = np.array([[0.0, 40e-6, 0.0]])
    E, _ = oracle.charge_field_lines(np.vstack([xyz, out]), np.concatenate([q, [1.6e-19]]), origin, step, shape)
    lines, nout = oracle.voxel_lines(xyz, q, origin, step, shape)
    ref = oracle.line_field(lines, out)[0, 1:]
    np.testing.assert_allclose(E[-1], ref, rtol=1e-12, atol=0)
