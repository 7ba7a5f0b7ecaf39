"""Pins of the oracle's Adaptive Modelling (Sec. 3: far copies of a periodic
structure with each primitive's average charge density): it reduces to the
exact sum when nothing is far or when the density is already uniform on
every primitive (the primitive's closed form is the sum of its elements'),
the averaged density keeps each primitive's charge, and the error falls as
more copies stay exact."""
import numpy as np

import oracle
from synth import strip_cell, uniform_points


def _setup(n_img=2):
    e, p, emap = strip_cell(n_img=n_img, sub_u=2, sub_w=4)
    pts = uniform_points(e.box_lo, e.box_hi, 40, 3)
    return e, p, emap, pts


def test_no_far_copies_is_exact():
    e, p, emap, pts = _setup()
    rng = np.random.default_rng(0)
    sigma = rng.standard_normal(e.n) * 1e-9
    ref = oracle.eval_points(e, sigma, pts)
    for k in (-1, 2, 5):
        np.testing.assert_array_equal(oracle.eval_adaptive(e, p, emap, k, sigma, pts), ref)


def test_uniform_density_per_primitive_is_exact():
    e, p, emap, pts = _setup()
    sig_p = np.array([1.0, -2.0, 0.5, 3.0, -1.5]) * 1e-9
    sigma = sig_p[emap]
    np.testing.assert_allclose(oracle.primitive_density(e, p, emap, sigma), sig_p, rtol=1e-14)
    ref = oracle.eval_points(e, sigma, pts)
    for k in (0, 1):
        got = oracle.eval_adaptive(e, p, emap, k, sigma, pts)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_charge_kept_and_error_falls_with_prim_after():
    e, p, emap, pts = _setup(n_img=3)
    rng = np.random.default_rng(1)
    sigma = (1.0 + 0.5 * rng.standard_normal(e.n)) * 1e-9
    sbar = oracle.primitive_density(e, p, emap, sigma)
    area = lambda g: np.linalg.norm(np.cross(g.u, g.w), axis=1)
    np.testing.assert_allclose(sbar * area(p), np.bincount(emap, sigma * area(e)), rtol=1e-13)
    ref = oracle.eval_points(e, sigma, pts)
    errs = [np.abs(oracle.eval_adaptive(e, p, emap, k, sigma, pts) - ref).max() for k in (0, 1, 2)]
    assert errs[0] > errs[1] > errs[2] > 0.0, errs
