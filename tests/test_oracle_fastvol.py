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


AXES = (np.array([-1.0e-3, -0.95e-3, -0.8e-3, -0.5e-3, 0.0, 0.9e-3]),
        np.array([0.5e-3, 0.51e-3, 0.6e-3, 1.25e-3]),
        np.array([2.0e-4, 2.02e-4, 2.1e-4, 2.5e-4, 4.0e-4]))


def test_graded_grid_nodes_linear_functions_and_uniform_case():
    rng = np.random.default_rng(3)
    nodes = oracle.axes_nodes(AXES)
    vals = rng.standard_normal((len(nodes), 4))
    np.testing.assert_allclose(oracle.trilinear_axes(AXES, vals, nodes), vals, rtol=0, atol=1e-12)
    # trilinear functions are reproduced on any cell sizes
    g = lambda p: ((1 + 1e3 * p[:, 0]) * (2 - 1e3 * p[:, 1]) * (0.5 + 3e3 * p[:, 2]))[:, None]
    lo = np.array([a[0] for a in AXES])
    hi = np.array([a[-1] for a in AXES])
    pts = rng.uniform(lo, hi, (500, 3))
    np.testing.assert_allclose(oracle.trilinear_axes(AXES, g(nodes), pts), g(pts), rtol=1e-12, atol=1e-12)
    # evenly spaced axes: the regular-grid interpolation
    ax = tuple(np.array(ORIGIN)[d] + np.arange(SHAPE[d]) * np.array(STEP)[d] for d in range(3))
    vals = rng.standard_normal((int(np.prod(SHAPE)), 2))
    pts = _pts(rng, 300)
    np.testing.assert_allclose(oracle.trilinear_axes(ax, vals, pts), oracle.trilinear(ORIGIN, STEP, SHAPE, vals, pts),
                               rtol=1e-12, atol=1e-12)


def test_graded_grid_quadratic_error_per_cell_and_outside():
    # f = x^2: at the midpoint of a cell of width h the error is h^2/4, with
    # h the width of that cell
    nodes = oracle.axes_nodes(AXES)
    vals = (nodes[:, 0] ** 2)[:, None]
    x = AXES[0]
    for c in range(len(x) - 1):
        h = x[c + 1] - x[c]
        mid = np.array([[0.5 * (x[c] + x[c + 1]), AXES[1][1], AXES[2][2]]])
        got = oracle.trilinear_axes(AXES, vals, mid)[0, 0]
        assert abs(got - (mid[0, 0] ** 2 + h * h / 4)) <= 1e-15, c
    out = np.array([[x[0] - 1e-9, AXES[1][0], AXES[2][0]], [x[0], AXES[1][0], AXES[2][-1] + 1e-9]])
    assert np.isnan(oracle.trilinear_axes(AXES, vals, out)).all()
    # the last node itself is inside (last cell, weight 1)
    last = np.array([[x[-1], AXES[1][-1], AXES[2][-1]]])
    assert oracle.trilinear_axes(AXES, vals, last)[0, 0] == x[-1] ** 2
