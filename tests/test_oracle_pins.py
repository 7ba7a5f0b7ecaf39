"""Pins for the CPU oracle: each checks it against something other than its
own formulas -- closed forms, independent quadrature, physical invariants.

Single-panel kernels (paper Sec. 2.1: Phi' = integral of 1/r over the panel,
E' = integral of r_hat / r^2):
  * square centroid and rectangle centre closed forms;
  * on-axis normal field over a square (solid angle);
  * triangle solid angle by the Van Oosterom-Strackee formula;
  * the 4 pi jump of the normal field and continuity of Phi' across a panel;
  * far-field monopole + quadrupole limit;
  * scaling (Phi' ~ length, E' scale-free);
  * rectangle = its two right triangles;
  * E' = -grad Phi' and Laplace's equation off the panel;
  * brute-force semi-analytic adaptive quadrature over random panels/points;
  * edge formula vs Gauss rule where both apply.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rand_panel(rng, kind, lx=None, lz=None):
    Q = _rot(rng)
    lx = rng.uniform(0.3, 2.0) if lx is None else lx
    lz = rng.uniform(0.3, 2.0) if lz is None else lz
    o = rng.standard_normal(3)
    return kind, o, lx * Q[:, 0], lz * Q[:, 1], Q, lx, lz


# ------------------------------------------------------------------ closed forms

def test_square_centroid_closed_form(oracle_lib):
    for L in (1.0, 62.5e-6, 3.0):
        o = np.array([-L / 2, -L / 2, 0.0])
        v = oracle.panel(0, o, [L, 0, 0], [0, L, 0], [0, 0, 0], on_plane=True)
        assert v[0] == pytest.approx(4 * L * math.log(1 + math.sqrt(2)), rel=2e-15)
        assert np.all(np.abs(v[1:]) <= 1e-14 * abs(v[0]) / L)


def test_rectangle_centre_closed_form(oracle_lib):
    # half sides p, q: 4 [p ln((q+d)/p) + q ln((p+d)/q)], d = sqrt(p^2+q^2)
    for p, q in ((1.0, 0.25), (0.3, 2.0), (1e-5, 3e-6)):
        d = math.hypot(p, q)
        ref = 4 * (p * math.log((q + d) / p) + q * math.log((p + d) / q))
        v = oracle.panel(0, [-p, -q, 0], [2 * p, 0, 0], [0, 2 * q, 0], [0, 0, 0], on_plane=True)
        assert v[0] == pytest.approx(ref, rel=4e-15)


def test_on_axis_normal_field_square(oracle_lib):
    a = 0.5
    for h in (1e-3, 0.1, 0.3, 1.0, 5.0, 40.0):
        ref = 4 * math.atan(a * a / (h * math.sqrt(2 * a * a + h * h)))
        v = oracle.panel(0, [-a, -a, 0], [2 * a, 0, 0], [0, 2 * a, 0], [0, 0, h])
        assert v[3] == pytest.approx(ref, rel=1e-13)
        assert abs(v[1]) < 1e-14 and abs(v[2]) < 1e-14
        # the potential on the axis: 4 h-integrated closed form via quad of the
        # on-axis normal field, Phi'(h) = integral_h^inf E'_n dh'
    # Phi' on the axis: integral of the normal field from h to infinity
    h = 0.3
    f = lambda t: 4 * math.atan(a * a / (t * math.sqrt(2 * a * a + t * t)))
    val, _ = integrate.quad(f, h, np.inf, epsabs=0, epsrel=2e-14, limit=200)
    v = oracle.panel(0, [-a, -a, 0], [2 * a, 0, 0], [0, 2 * a, 0], [0, 0, h])
    assert v[0] == pytest.approx(val, rel=1e-12)


def test_triangle_solid_angle_van_oosterom_strackee(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(300):
        kind, o, u, w, Q, lx, lz = _rand_panel(rng, 1)
        n = np.cross(u, w) / np.linalg.norm(np.cross(u, w))
        p = o + rng.uniform(-3, 3, 3)
        r1, r2, r3 = p - o, p - (o + u), p - (o + w)
        a1, a2, a3 = (np.linalg.norm(x) for x in (r1, r2, r3))
        num = np.dot(r1, np.cross(r2, r3))
        den = a1 * a2 * a3 + np.dot(r1, r2) * a3 + np.dot(r1, r3) * a2 + np.dot(r2, r3) * a1
        omega = 2 * math.atan2(num, den)
        v = oracle.panel(1, o, u, w, p)
        assert np.dot(v[1:], n) == pytest.approx(omega, rel=1e-11, abs=1e-13)


def test_normal_field_jump_and_potential_continuity(oracle_lib):
    rng = np.random.default_rng(5)
    for kind in (0, 1):
        for _ in range(20):
            k, o, u, w, Q, lx, lz = _rand_panel(rng, kind)
            n = np.cross(u, w) / np.linalg.norm(np.cross(u, w))
            s, t = rng.uniform(0.1, 0.4, 2)
            x = o + s * u + t * w
            eps = 1e-9
            vp = oracle.panel(kind, o, u, w, x + eps * n)
            vm = oracle.panel(kind, o, u, w, x - eps * n)
            v0 = oracle.panel(kind, o, u, w, x, on_plane=True)
            jump = np.dot(vp[1:] - vm[1:], n)
            assert jump == pytest.approx(4 * math.pi, rel=1e-7)
            assert vp[0] == pytest.approx(vm[0], rel=1e-7)
            assert v0[0] == pytest.approx(0.5 * (vp[0] + vm[0]), rel=1e-7)
            assert abs(np.dot(v0[1:], n)) < 1e-13 * np.linalg.norm(vp[1:])  # principal value


def test_far_field_monopole_quadrupole(oracle_lib):
    rng = np.random.default_rng(7)
    lx, lz = 1.0, 0.6
    o = np.array([-lx / 2, -lz / 2, 0.0])
    area = lx * lz
    for R in (20.0, 60.0, 200.0):
        for _ in range(5):
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            p = R * d
            v = oracle.panel(0, o, [lx, 0, 0], [0, lz, 0], p)
            quad = area * (lx**2 * (3 * d[0]**2 - 1) + lz**2 * (3 * d[1]**2 - 1)) / (24 * R**3)
            mono = area / R
            # next (hexadecapole) term is O(area * D^4 / R^5)
            assert abs(v[0] - mono - quad) <= 0.2 * area * (lx**2 + lz**2)**2 / R**5
            Emono = area * p / R**3
            assert np.linalg.norm(v[1:] - Emono) <= 2.0 * area * (lx**2 + lz**2) / R**4


def test_scaling(oracle_lib):
    rng = np.random.default_rng(3)
    for kind in (0, 1):
        k, o, u, w, Q, lx, lz = _rand_panel(rng, kind)
        p = o + rng.uniform(-2, 2, 3)
        v = oracle.panel(kind, o, u, w, p)
        for lam in (1e-5, 7.0):
            vs = oracle.panel(kind, lam * o, lam * u, lam * w, lam * p)
            assert vs[0] == pytest.approx(lam * v[0], rel=1e-13)
            np.testing.assert_allclose(vs[1:], v[1:], rtol=1e-12, atol=1e-13 * np.abs(v[1:]).max())


def test_rectangle_is_two_right_triangles(oracle_lib):
    rng = np.random.default_rng(9)
    for _ in range(200):
        k, o, u, w, Q, lx, lz = _rand_panel(rng, 0)
        p = o + rng.uniform(-3, 3, 3) * 0.5 * (lx + lz)
        r = oracle.panel(0, o, u, w, p, method="exact")
        t1 = oracle.panel(1, o, u, w, p, method="exact")
        t2 = oracle.panel(1, o + u + w, -u, -w, p, method="exact")
        np.testing.assert_allclose(r, t1 + t2, rtol=1e-12, atol=1e-13 * np.abs(r).max())


def _fd_grad(f, p, h):
    g = np.zeros(3)
    for k in range(3):
        d = np.zeros(3)
        d[k] = h
        g[k] = (8 * (f(p + d) - f(p - d)) - (f(p + 2 * d) - f(p - 2 * d))) / (12 * h)
    return g


def test_field_is_minus_gradient_and_harmonic(oracle_lib):
    rng = np.random.default_rng(13)
    for kind in (0, 1):
        for _ in range(10):
            k, o, u, w, Q, lx, lz = _rand_panel(rng, kind)
            n = np.cross(u, w) / np.linalg.norm(np.cross(u, w))
            p = o + 0.5 * (u + w) + rng.uniform(0.3, 1.5) * n + rng.uniform(-1, 1, 3) * 0.5
            f = lambda x: oracle.panel(kind, o, u, w, x)[0]
            g = _fd_grad(f, p, 1e-3)
            v = oracle.panel(kind, o, u, w, p)
            np.testing.assert_allclose(v[1:], -g, rtol=1e-8, atol=1e-9 * np.abs(v[1:]).max())
            # Laplace's equation off the panel: div E' = 0 (4th-order differences)
            div = sum(_fd_grad(lambda x, k=k: oracle.panel(kind, o, u, w, x)[1 + k], p, 3e-4)[k]
                      for k in range(3))
            assert abs(div) < 1e-8 * np.linalg.norm(v[1:])


# --------------------------------------------------------- brute-force quadrature

def _semi_analytic(kind, lx, lz, X, h, Z):
    """Phi', E' of the canonical panel (corner at 0, edges along local x, z)
    at the local point (X, h, Z): the x-integral in closed form (antiderivatives
    of 1/r, (X-x)/r^3 and 1/r^3), the z-integral by adaptive Gauss-Kronrod."""
    def xmax(z):
        return lx if kind == 0 else lx * (1.0 - z / lz)

    def inner(z, comp):
        c2 = h * h + (Z - z) ** 2
        a1, a2 = X - 0.0, X - xmax(z)
        r1, r2 = math.sqrt(a1 * a1 + c2), math.sqrt(a2 * a2 + c2)
        if comp == 0:
            return math.asinh(a1 / math.sqrt(c2)) - math.asinh(a2 / math.sqrt(c2))
        if comp == 1:  # E'_x
            return 1.0 / r2 - 1.0 / r1
        g = (-a2 / (c2 * r2)) - (-a1 / (c2 * r1))  # integral of dx / r^3
        return (Z - z) * g if comp == 3 else h * g

    out = []
    pts = [Z] if 0 < Z < lz else None
    for comp in range(4):
        val, err = integrate.quad(inner, 0.0, lz, args=(comp,), epsabs=0, epsrel=2e-14, limit=400,
                                  points=pts)
        out.append(val)
    return np.array(out)  # Phi', E'x (local), E'h (normal), E'z (local)


@pytest.mark.parametrize("kind", [0, 1])
def test_bruteforce_adaptive_quadrature(oracle_lib, kind):
    rng = np.random.default_rng(100 + kind)
    worst = 0.0
    for i in range(150):
        k, o, u, w, Q, lx, lz = _rand_panel(rng, kind)
        # distances from 0.02 D to 30 D, a third of them almost on the plane
        D = math.hypot(lx, lz)
        X = rng.uniform(-1.0, 2.0) * lx
        Z = rng.uniform(-1.0, 2.0) * lz
        h = (rng.uniform(0.02, 1.0) if i % 3 else rng.uniform(0.01, 0.05)) * D * rng.choice([-1, 1])
        if i % 10 == 0:
            X, Z, h = X * 20, Z * 20, h * 10
        ref = _semi_analytic(kind, lx, lz, X, h, Z)
        n = Q[:, 2] if np.dot(np.cross(u, w), Q[:, 2]) > 0 else -Q[:, 2]
        p = o + X * Q[:, 0] + Z * Q[:, 1] + h * n
        v = oracle.panel(kind, o, u, w, p)
        loc = np.array([v[0], np.dot(v[1:], Q[:, 0]), np.dot(v[1:], n), np.dot(v[1:], Q[:, 1])])
        scale = np.abs(ref[1:]).max()
        err = max(abs(loc[0] - ref[0]) / abs(ref[0]), np.abs(loc[1:] - ref[1:]).max() / scale)
        worst = max(worst, err)
    assert worst < 1e-12, worst


def test_edge_formula_matches_gauss_rule(oracle_lib):
    rng = np.random.default_rng(21)
    for kind in (0, 1):
        for _ in range(100):
            k, o, u, w, Q, lx, lz = _rand_panel(rng, kind)
            D = math.hypot(lx, lz)
            c = o + (0.5 if kind == 0 else 1 / 3) * (u + w)
            d = rng.standard_normal(3)
            p = c + rng.uniform(8, 30) * D * d / np.linalg.norm(d)
            e = oracle.panel(kind, o, u, w, p, method="exact")
            g = oracle.panel(kind, o, u, w, p, method="gauss")
            np.testing.assert_allclose(e, g, rtol=5e-13, atol=5e-13 * np.abs(g).max())
