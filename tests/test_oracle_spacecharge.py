"""Pins for the oracle's space-charge pieces, from physics rather than from the
oracle's own formulas:

  * the right-hand side with known charges (Sec. 4.1, RHVector with the
    known-charge share; Algorithm 2's sum at the collocation points):
      - conductor rows: a point charge between two grounded plates induces
        -q (1 - z0/d) on the plate it is z0 from and -q z0/d on the other
        (Green's reciprocity), and the total potential vanishes on both;
      - interface rows: a sheet of charges above a flat periodic dielectric
        interface binds sigma_b = -(eps - 1)/(eps + 1) times the charge
        sheet's normal field at the interface in units of sigma_f/(2 eps0)
        (the normal displacement is continuous; a flat sheet adds no normal
        field in its own plane);
  * the explicit move of the dynamic loop (Algorithm 4): a lone ion in the
    parallel-plate field moves along E, an electron against it, by
    mobility |E| dt;
  * the point-to-line reduction (Algorithm 3): a voxel holding charges of
    both signs, placed by hand, for both placements.
"""
import numpy as np
import pytest

import oracle
from synth import GeometryBuilder, Images, parallel_plates
from synth.geometry import DIELECTRIC

E = 1.602176634e-19


@pytest.fixture(scope="module")
def grounded_plates(oracle_lib):
    # 2 mm plates 0.2 mm apart: a charge's field dies off as exp(-pi r/d)
    # along the gap, so the plates act as infinite ones for the induced charge
    g = parallel_plates(n=40, side=2e-3, gap=0.2e-3, v_bottom=0.0, v_top=0.0)
    return g, oracle.assemble(g)


@pytest.mark.parametrize("frac", [0.3, 0.5, 0.8])
def test_rhs_with_charges_induced_charge_on_grounded_plates(grounded_plates, frac):
    g, A = grounded_plates
    d = 0.2e-3
    h = 2e-3 / 40
    z0 = -d / 2 + frac * d
    qxyz = np.array([[0.37 * h, 0.21 * h, z0]])
    b = oracle.rhs_with_charges(g, g.rhs(), qxyz, np.array([E]))
    s = oracle.solve(A, b)
    Q = s * g.areas()
    half = g.n // 2  # bottom plate first
    assert Q[:half].sum() / E == pytest.approx(-(1.0 - frac), abs=2e-4)
    assert Q[half:].sum() / E == pytest.approx(-frac, abs=2e-4)
    # the total potential (panels + charge) vanishes at every collocation point
    phi = oracle.eval_points(g, s, g.centroids())[:, 0] + oracle.coulomb(g.centroids(), qxyz, [E])[:, 0]
    assert np.abs(phi).max() <= 1e-10 * np.abs(oracle.coulomb(g.centroids(), qxyz, [E])[:, 0]).max()


def test_rhs_with_charges_bound_charge_on_dielectric_interface(oracle_lib):
    a, npan, K, eps = 50e-6, 2, 8, 4.0
    b = GeometryBuilder()
    hp = a / npan
    for i in range(npan):
        for j in range(npan):
            b.rect((i * hp, j * hp, 0.0), (hp, 0, 0), (0, hp, 0), bc=DIELECTRIC, eps_pos=1.0, eps_neg=eps)
    g = b.build("interface", Images(a1=np.array([a, 0.0, 0.0]), a2=np.array([0.0, a, 0.0]), n1=K, n2=K),
                (0, 0, -a), (a, a, a))
    A = oracle.assemble(g)
    # charges on a 5 um grid at 10 um above the interface, over the copies'
    # whole extent: a sheet of density sigma_f = e / s^2 on the +n side
    hq, s = 10e-6, 5e-6
    lo, ext = -K * a, (2 * K + 1) * a
    xs = lo + s / 2 + s * np.arange(int(round(ext / s)))
    X, Y = np.meshgrid(xs, xs)
    qxyz = np.column_stack([X.ravel(), Y.ravel(), np.full(X.size, hq)])
    sigma_f = E / s ** 2
    rhs = oracle.rhs_with_charges(g, g.rhs(), qxyz, np.full(X.size, E))
    sb = oracle.solve(A, rhs)
    # the sheet's normal field at each collocation point, from the closed form
    # of a uniformly charged square of the same extent (field k_e sigma_f E'),
    # as a fraction f of the infinite sheet's sigma_f / (2 eps0)
    f = np.array([-oracle.panel(0, (lo, lo, hq), (ext, 0, 0), (0, ext, 0), c)[3] / (2 * np.pi)
                  for c in g.centroids()])
    assert np.all((f > 0.9) & (f < 1.0))
    np.testing.assert_allclose(sb / sigma_f, -(eps - 1.0) / (eps + 1.0) * f, rtol=1e-4)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_spacecharge_move_along_field(oracle_lib, sign):
    g = parallel_plates()  # bottom 0 V at z = -0.1 mm, top 1 V at z = +0.1 mm
    A = oracle.assemble(g)
    b0 = g.rhs()
    s0 = oracle.solve(A, b0)
    x0 = np.array([[0.3e-6, -0.2e-6, 0.01e-3]])
    p = oracle.SpaceChargeParams(dt=1e-12, mobility=1e-4, resolve_every=10)
    new, sigma, Ef = oracle.spacecharge_step(g, A, b0, s0, x0, np.array([sign * E]), 0, p)
    E_plates = oracle.eval_points(g, s0, x0)[0, 1:]
    # between the plates the field points from the 1 V plate to the 0 V one
    assert E_plates[2] < 0 and 4000.0 < np.linalg.norm(E_plates) < 6000.0
    # the charge's own image charges change E by a few 1e-6 of the plates' field
    assert np.linalg.norm(Ef[0] - E_plates) <= 1e-5 * np.linalg.norm(E_plates)
    disp = new[0] - x0[0]
    step = sign * p.mobility * p.dt * E_plates
    assert np.linalg.norm(disp - step) <= 1e-5 * np.linalg.norm(step)
    assert np.sign(disp[2]) == -sign  # ion towards the 0 V plate, electron towards the 1 V one


def test_voxel_placement_mixed_sign_voxel(oracle_lib):
    origin, step, shape = (0.0, 0.0, 0.0), (5e-6, 5e-6, 5e-6), (4, 4, 4)
    # voxel (1, 2, 0): +2e at offset (1, 1) um, -e at offset (4, 3) um
    base = np.array([5e-6, 10e-6, 0.0])
    xyz = base + np.array([[1e-6, 1e-6, 2e-6], [4e-6, 3e-6, 1e-6]])
    q = np.array([2 * E, -E])
    for placement, (ex, ey) in (("centre", (2.5e-6, 2.5e-6)), ("weighted", (2e-6, 5e-6 / 3))):
        lines, out = oracle.voxel_lines(xyz, q, origin, step, shape, placement=placement)
        assert out == 0 and lines.shape == (1, 7)
        x, y = lines[0, 0] - base[0], lines[0, 1] - base[1]
        assert x == pytest.approx(ex, rel=1e-12) and y == pytest.approx(ey, rel=1e-12)
        # inside its own voxel, one voxel tall, the voxel's net charge
        assert 0.0 <= x < step[0] and 0.0 <= y < step[1]
        assert (lines[0, 2], lines[0, 5]) == (0.0, step[2])
        assert lines[0, 6] * step[2] == pytest.approx(E, rel=1e-12)


def test_spacecharge_threshold_rule(oracle_lib):
    """Algorithm 4's SpChTh: with a threshold the re-solve happens exactly
    when the charges' magnitude sum |q| exceeds it -- a neutral +-e pair
    counts 2e, not 0 -- and the fixed schedule is not consulted."""
    g = parallel_plates(n=6)
    A = oracle.assemble(g)
    b0 = g.rhs()
    s0 = oracle.solve(A, b0)
    x = np.array([[0.1e-3, 0.0, 0.02e-3], [-0.1e-3, 0.05e-3, -0.03e-3]])
    q = np.array([E, -E])
    for thr, due in ((1.5 * E, True), (2.5 * E, False)):
        p = oracle.SpaceChargeParams(threshold=thr, resolve_every=1)
        _, sigma, _ = oracle.spacecharge_step(g, A, b0, s0, x, q, 0, p)
        assert (not np.array_equal(sigma, s0)) == due
        p = oracle.SpaceChargeParams(threshold=thr, resolve_every=10)
        _, sigma, _ = oracle.spacecharge_step(g, A, b0, s0, x, q, 3, p)  # off-schedule step
        assert (not np.array_equal(sigma, s0)) == due
