"""Pins of the oracle's FastVolume interpolation (trilinear on a regular
grid, the paper's Sec. 3 volume sampling): node values come back exactly,
any function linear in x, y, z and any product of three linear factors
(the trilinear space itself) is reproduced exactly inside the grid, and
points outside give NaN."""
import numpy as np

import oracle

ORIGIN, STEP, SHAPE = (-1.0e-3, 0.5e-3, 2.0e-4), (1.0e-4, 2.5e-4, 5.0e-5), (7, 4, 5)


def _pts(rng, m):
    lo = np.array(ORIGIN)
    hi = lo + (np.array(SHAPE) - 1) * np.array(STEP)
    return rng.uniform(lo, hi, (m, 3))


def test_nodes_exact():
    rng = np.random.default_rng(0)
    nodes = oracle.grid_nodes(ORIGIN, STEP, SHAPE)
    vals = rng.standard_normal((len(nodes), 4))
    got = oracle.trilinear(ORIGIN, STEP, SHAPE, vals, nodes)
    np.testing.assert_allclose(got, vals, rtol=0, atol=1e-12)


def test_trilinear_functions_reproduced():
    rng = np.random.default_rng(1)
    nodes = oracle.grid_nodes(ORIGIN, STEP, SHAPE)
    a = rng.standard_normal((4, 4))
    f = lambda p: np.column_stack([a[c, 0] + a[c, 1] * p[:, 0] * 1e3 + a[c, 2] * p[:, 1] * 1e3
                                   + a[c, 3] * p[:, 2] * 1e3 for c in range(4)])
    g = lambda p: ((1 + 1e3 * p[:, 0]) * (2 - 1e3 * p[:, 1]) * (0.5 + 3e3 * p[:, 2]))[:, None]
    pts = _pts(rng, 500)
    np.testing.assert_allclose(oracle.trilinear(ORIGIN, STEP, SHAPE, f(nodes), pts), f(pts), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.trilinear(ORIGIN, STEP, SHAPE, g(nodes), pts), g(pts), rtol=1e-12, atol=1e-12)


def test_quadratic_error_bound_and_outside():
    # f = x^2 along x: trilinear error at a cell's midpoint is h^2/4 exactly
    h = STEP[0]
    nodes = oracle.grid_nodes(ORIGIN, STEP, SHAPE)
    vals = (nodes[:, 0] ** 2)[:, None]
    mid = np.array([[ORIGIN[0] + 2.5 * h, ORIGIN[1] + STEP[1], ORIGIN[2] + STEP[2]]])
    got = oracle.trilinear(ORIGIN, STEP, SHAPE, vals, mid)[0, 0]
    assert abs(got - (mid[0, 0] ** 2 + h * h / 4)) <= 1e-15
    out = np.array([[ORIGIN[0] - 1e-9, ORIGIN[1], ORIGIN[2]],
                    [ORIGIN[0], ORIGIN[1] + (SHAPE[1] - 1) * STEP[1] * (1 + 1e-9), ORIGIN[2]]])
    assert np.isnan(oracle.trilinear(ORIGIN, STEP, SHAPE, vals, out)).all()
