"""Pins for the oracle's assembled system, solve, evaluation and point-charge
sums (paper Eq. Matrix, Eqs. Potential/Field, Sec. 3 periodic copies,
Algorithm 2's charge sum), against invariants and closed forms:

  * parallel plates: A = A^T, the diagonal's closed form, D4 symmetry of
    sigma, superposition, capacitance above the ideal value;
  * evaluation rows equal assembly rows (conductor potential is continuous);
  * selected rows (assemble_rows) equal the full assembly's, conductor and
    interface rows, with copies;
  * Gauss's law on a closed box around part of the panels;
  * lattice copies equal explicitly translated panels;
  * mirror copies: antisymmetric -> phi = 0 on the plane, symmetric -> E_n = 0;
  * far points: phi -> k_e Q / R;
  * dielectric interface rows: two-layer capacitor limit;
  * point charges: two-charge closed form, sum q_i E_i = 0, neutral pairs.
"""
import math
import warnings

import numpy as np
import pytest

import oracle
from synth import GeometryBuilder, Images, gem_cell, parallel_plates, uniform_points
from synth.geometry import CONDUCTOR, DIELECTRIC

warnings.filterwarnings("ignore", category=UserWarning)


@pytest.fixture(scope="module")
def plates(oracle_lib):
    g = parallel_plates()
    A = oracle.assemble(g)
    return g, A


def test_plates_matrix_symmetric_and_diagonal(plates):
    g, A = plates
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    h = 62.5e-6
    diag = oracle.ke() * 4 * h * math.log(1 + math.sqrt(2))
    np.testing.assert_allclose(np.diag(A), diag, rtol=2e-15)
    assert diag == pytest.approx(1.98034769e6, rel=1e-8)


def test_plates_sigma_symmetry_superposition_capacitance(plates):
    g, A = plates
    b = g.rhs()
    s = oracle.solve(A, b)
    # backward error at rounding level
    assert np.linalg.norm(A @ s - b) <= 1e-13 * np.linalg.norm(A, 2) * np.linalg.norm(s)
    # D4 symmetry of each plate's 16x16 grid
    for p in range(2):
        m = s[p * 256:(p + 1) * 256].reshape(16, 16)
        for t in (m.T, m[::-1, :], m[:, ::-1], np.rot90(m)):
            np.testing.assert_allclose(t, m, rtol=1e-12)
    # superposition: sigma(1,0) = (sigma(1,1) + sigma(1,-1)) / 2
    bt = np.where(np.arange(512) < 256, 1.0, 1.0)
    ba = np.where(np.arange(512) < 256, -1.0, 1.0)
    np.testing.assert_allclose(s, 0.5 * (oracle.solve(A, bt) + oracle.solve(A, ba)), rtol=1e-11,
                               atol=1e-12 * np.abs(s).max())
    # antisymmetric drive: potential zero on the mid-plane
    sa = oracle.solve(A, 0.5 * ba)
    mid = uniform_points((-0.5e-3, -0.5e-3, 0.0), (0.5e-3, 0.5e-3, 0.0), 64, 4)
    f = oracle.eval_points(g, sa, mid)
    assert np.abs(f[:, 0]).max() < 1e-12
    # capacitance exceeds the ideal (fringing) value eps0 A / d
    area = g.areas()
    q_top = np.sum(s[256:] * area[256:])
    c_ideal = oracle.eps0() * 1e-6 / 0.2e-3
    assert 1.0 < q_top / c_ideal < 2.0


def test_eval_equals_assembly_rows(plates):
    g, A = plates
    s = oracle.solve(A, g.rhs())
    c = g.centroids()
    f = oracle.eval_points(g, s, c)
    np.testing.assert_allclose(f[:, 0], g.rhs(), rtol=0, atol=1e-11)


def test_assemble_rows_equal_full_assembly(oracle_lib):
    """The row-subset entry point (used where the full matrix is out of
    reach) gives exactly the full assembly's rows, for conductor and
    dielectric-interface rows with periodic copies."""
    g = gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2)
    A = oracle.assemble(g)
    rows = np.concatenate([[0, g.n // 2, g.n - 1],
                           np.random.default_rng(3).choice(g.n, 9, replace=False)])
    assert {CONDUCTOR, DIELECTRIC} <= set(np.asarray(g.bc)[rows].tolist())  # both row kinds present
    R = oracle.assemble_rows(g, rows)
    assert np.array_equal(R, A[rows])


def _small_mixed_geometry(rng):
    """A few rectangles and right triangles at random orientations."""
    b = GeometryBuilder()
    for i in range(6):
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        o = rng.uniform(-1e-3, 1e-3, 3)
        lx, lz = rng.uniform(0.2e-3, 0.6e-3, 2)
        if i % 2:
            b.rect(o, lx * q[:, 0], lz * q[:, 1])
        else:
            b.right_tri(o, lx * q[:, 0], lz * q[:, 1])
    return b.build("mixed", Images(), (-2e-3,) * 3, (2e-3,) * 3)


def _box_flux(g, sigma, lo, hi, nsub=6, m=10):
    """Outward flux of E through the box [lo, hi] by composite Gauss-Legendre."""
    x, wq = np.polynomial.legendre.leggauss(m)
    x, wq = 0.5 * (x + 1), 0.5 * wq
    total = 0.0
    for ax in range(3):
        a1, a2 = [k for k in range(3) if k != ax]
        for side, sgn in ((lo[ax], -1.0), (hi[ax], 1.0)):
            pts, wts = [], []
            la = (hi[a1] - lo[a1]) / nsub
            lb = (hi[a2] - lo[a2]) / nsub
            for i in range(nsub):
                for j in range(nsub):
                    for p in range(m):
                        for q in range(m):
                            r = np.empty(3)
                            r[ax] = side
                            r[a1] = lo[a1] + (i + x[p]) * la
                            r[a2] = lo[a2] + (j + x[q]) * lb
                            pts.append(r)
                            wts.append(wq[p] * wq[q] * la * lb)
            f = oracle.eval_points(g, sigma, np.array(pts))
            total += sgn * np.dot(np.array(wts), f[:, 1 + ax])
    return total


def test_gauss_law_closed_box(oracle_lib):
    rng = np.random.default_rng(17)
    g = _small_mixed_geometry(rng)
    sigma = rng.uniform(-1e-6, 1e-6, g.n)
    # box enclosing all panels, faces well away from them
    lo = np.array([-2.5e-3] * 3)
    hi = np.array([2.5e-3] * 3)
    flux = _box_flux(g, sigma, lo, hi)
    q = np.sum(sigma * g.areas())
    assert flux == pytest.approx(q / oracle.eps0(), rel=1e-10)
    # a box containing none of them: zero flux
    lo2 = np.array([3e-3, 3e-3, 3e-3])
    hi2 = np.array([4e-3, 4e-3, 4e-3])
    assert abs(_box_flux(g, sigma, lo2, hi2, nsub=3)) < 1e-10 * abs(q) / oracle.eps0()


def test_far_points_monopole(oracle_lib):
    rng = np.random.default_rng(19)
    g = _small_mixed_geometry(rng)
    sigma = rng.uniform(0.5e-6, 1e-6, g.n)
    q = np.sum(sigma * g.areas())
    cm = np.sum((sigma * g.areas())[:, None] * g.centroids(), axis=0) / q
    d = rng.standard_normal((8, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = cm + 10.0 * d  # 10 m away from a mm-sized cluster
    f = oracle.eval_points(g, sigma, pts)
    np.testing.assert_allclose(f[:, 0], oracle.ke() * q / 10.0, rtol=1e-7)


def test_lattice_copies_equal_translated_panels(oracle_lib):
    rng = np.random.default_rng(23)
    g = _small_mixed_geometry(rng)
    sigma = rng.uniform(-1e-6, 1e-6, g.n)
    im = Images(a1=np.array([3e-3, 0, 0]), a2=np.array([1e-3, 2.5e-3, 0]), n1=1, n2=2)
    gi = g.with_images(im)
    t = im.translations()
    b = GeometryBuilder()
    for tk in t:
        for j in range(g.n):
            (b.rect if g.kind[j] == 0 else b.right_tri)(g.o[j] + tk, g.u[j], g.w[j])
    ge = b.build("explicit", Images(), g.box_lo, g.box_hi)
    pts = uniform_points((-2e-3,) * 3, (2e-3,) * 3, 50, 5)
    f1 = oracle.eval_points(gi, sigma, pts)
    f2 = oracle.eval_points(ge, np.tile(sigma, len(t)), pts)
    np.testing.assert_allclose(f1, f2, rtol=1e-12, atol=1e-12 * np.abs(f2).max())


def test_mirror_copies(oracle_lib):
    rng = np.random.default_rng(29)
    g = _small_mixed_geometry(rng)
    g.o[:, 2] += 3e-3  # all panels above z = 0
    sigma = rng.uniform(-1e-6, 1e-6, g.n)
    on_plane = uniform_points((-3e-3, -3e-3, 0.0), (3e-3, 3e-3, 0.0), 40, 6)
    anti = g.with_images(Images(mirror_mask=4, mirror_pos=np.zeros(3),
                                mirror_parity=np.array([1, 1, -1], dtype=np.int32)))
    f = oracle.eval_points(anti, sigma, on_plane)
    scale = np.abs(oracle.eval_points(g, sigma, on_plane)[:, 0]).max()
    assert np.abs(f[:, 0]).max() <= 1e-13 * scale
    sym = g.with_images(Images(mirror_mask=4, mirror_pos=np.zeros(3),
                               mirror_parity=np.array([1, 1, 1], dtype=np.int32)))
    f = oracle.eval_points(sym, sigma, on_plane)
    assert np.abs(f[:, 3]).max() <= 1e-12 * np.abs(f[:, 1:3]).max()
    # a mirror copy equals the explicitly reflected panel
    b = GeometryBuilder()
    for j in range(g.n):
        (b.rect if g.kind[j] == 0 else b.right_tri)(g.o[j], g.u[j], g.w[j])
    for j in range(g.n):
        flip = np.array([1.0, 1.0, -1.0])
        (b.rect if g.kind[j] == 0 else b.right_tri)(g.o[j] * flip, g.u[j] * flip, g.w[j] * flip)
    ge = b.build("explicit", Images(), g.box_lo, g.box_hi)
    pts = uniform_points((-2e-3,) * 3, (2e-3,) * 3, 30, 7)
    f1 = oracle.eval_points(anti, sigma, pts)
    f2 = oracle.eval_points(ge, np.concatenate([sigma, -sigma]), pts)
    np.testing.assert_allclose(f1, f2, rtol=1e-12, atol=1e-12 * np.abs(f2).max())


def test_dielectric_interface_two_layer_capacitor(oracle_lib):
    """Plates at z = -g/2 (0 V) and +g/2 (V); dielectric eps_r below z = 0,
    vacuum above; periodic cell copies make the plates nearly infinite.
    Infinite-capacitor limit: E_below = 2V/(g(1+eps_r)), interface density
    sigma = eps0 (E_z(above) - E_z(below)) = 2 eps0 V (1-eps_r)/(g(1+eps_r))."""
    cell, gap, V, er, n = 1e-3, 0.1e-3, 1.0, 4.0, 4
    b = GeometryBuilder()
    h = cell / n
    for z, kind in ((-gap / 2, "bot"), (0.0, "int"), (gap / 2, "top")):
        for i in range(n):
            for j in range(n):
                o = (i * h, j * h, z)
                if kind == "int":
                    b.rect(o, (h, 0, 0), (0, h, 0), bc=DIELECTRIC, eps_pos=1.0, eps_neg=er)
                else:
                    b.rect(o, (h, 0, 0), (0, h, 0), bc=CONDUCTOR, value=(V if kind == "top" else 0.0))
    im = Images(a1=np.array([cell, 0, 0]), a2=np.array([0, cell, 0]), n1=20, n2=20)
    g = b.build("two_layer", im, (0, 0, -gap), (cell, cell, gap))
    A = oracle.assemble(g)
    s = oracle.solve(A, g.rhs())
    s_int = s[n * n:2 * n * n]
    ref = 2 * oracle.eps0() * V * (1 - er) / (gap * (1 + er))
    np.testing.assert_allclose(s_int, ref, rtol=5e-3)
    s_top = s[2 * n * n:]
    # free charge on the top plate: D = eps0 * E_above
    e_above = er * 2 * V / (gap * (1 + er))
    np.testing.assert_allclose(s_top, oracle.eps0() * e_above, rtol=5e-3)


def test_point_charges(oracle_lib):
    ke = oracle.ke()
    # two charges: closed form
    src = np.array([[0.0, 0.0, 0.0], [1e-5, 2e-5, -1e-5]])
    q = np.array([1e-18, -3e-18])
    f = oracle.coulomb(src, src, q, self_index=np.arange(2))
    r = src[0] - src[1]
    rr = np.linalg.norm(r)
    assert f[0, 0] == pytest.approx(ke * q[1] / rr, rel=1e-15)
    np.testing.assert_allclose(f[0, 1:], ke * q[1] * r / rr**3, rtol=1e-15)
    # Newton's third law on a random cloud: sum_i q_i E_i = 0
    rng = np.random.default_rng(31)
    xyz = rng.standard_normal((300, 3)) * 2e-5
    qq = np.where(np.arange(300) % 2 == 0, 1.6e-19, -1.6e-19)
    f = oracle.coulomb(xyz, xyz, qq, self_index=np.arange(300))
    force = (qq[:, None] * f[:, 1:]).sum(axis=0)
    scale = np.abs(qq[:, None] * f[:, 1:]).sum()
    assert np.abs(force).max() <= 1e-14 * scale
    # neutral cloud of coincident +- pairs: zero field at outside points
    pair = np.repeat(xyz[:50], 2, axis=0)
    qp = np.tile([1.6e-19, -1.6e-19], 50)
    tgt = rng.standard_normal((20, 3)) * 1e-4
    f = oracle.coulomb(tgt, pair, qp)
    assert np.abs(f).max() <= 1e-14 * ke * 1.6e-19 * 50 / 1e-8


def test_refined_solve_residual_and_agreement():
    """Iterative refinement keeps the solution of the same system and brings
    an ill-conditioned system's residual down to rounding."""
    rng = np.random.default_rng(12)
    n = 300
    U_, _ = np.linalg.qr(rng.normal(size=(n, n)))
    V_, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = (U_ * np.logspace(0, -9, n)) @ V_.T  # condition number 1e9
    x_true = rng.normal(size=n)
    b = A @ x_true
    x0 = oracle.solve(A, b)
    x1 = oracle.solve_refined(A, b)
    r0 = np.linalg.norm(b - A @ x0)
    r1 = np.linalg.norm(b - A @ x1)
    assert r1 <= r0 and r1 <= 1e-15 * np.linalg.norm(A, 2) * np.linalg.norm(x1) * n
    # both within the conditioning bound of the true solution
    assert np.linalg.norm(x1 - x_true) <= 1e9 * 1e-13 * np.linalg.norm(x_true)
