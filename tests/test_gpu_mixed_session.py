"""Mixed-precision path, resident sessions and the space-charge step on the
GPU, against the CPU oracle.

Bars: FP64 path 1e-10 relative; mixed path 1e-6 relative (phi and E,
pointwise on points where the reference is >= 1e-3 of its maximum); the
mixed solve must reach ||b - A x|| <= 1e-10 ||b||.  Point-charge sums run in
FP32 per pair with FP64 accumulation: their error is bounded relative to the
sum of the absolute pair terms (condition-normalised) by 1e-6.
"""
import math

import numpy as np
import pytest

import oracle
from synth import GeometryBuilder, Images, charge_cloud, gem_cell, gem_eval_points, uniform_points

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def nb():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2606_24154_amd as nb
    return nb


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def cols(pts):
    return [dev(pts[:, k]) for k in range(3)]


def stack(out):
    torch.cuda.synchronize()
    return np.column_stack([t.cpu().numpy() for t in out])


def rel_errors(got, ref, floor=1e-3):
    ap = np.abs(ref[:, 0])
    sel = ap >= floor * ap.max()
    ephi = np.max(np.abs(got[sel, 0] - ref[sel, 0]) / ap[sel])
    en = np.linalg.norm(ref[:, 1:], axis=1)
    sel = en >= floor * en.max()
    eE = np.max(np.linalg.norm(got[sel, 1:] - ref[sel, 1:], axis=1) / en[sel])
    return ephi, eE


@pytest.fixture(scope="module")
def small_gem():
    """Reduced GEM cell (688 elements, 25 copies) for full-pipeline parity."""
    g = gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2)
    A = oracle.assemble(g)
    s = oracle.solve(A, g.rhs())
    pts = gem_eval_points(g, 600, seed=11)
    f = oracle.eval_points(g, s, pts)
    return g, A, s, pts, f


# ----------------------------------------------------------------- mixed eval

@pytest.mark.parametrize("kind", [0, 1])
def test_mixed_single_element_far_field(nb, kind):
    """FP64 monopole + FP32 quadrature correction at R >= 4 D: <= 5e-7 per
    element copy; exact FP64 below 4 D (<= 1e-10)."""
    rng = np.random.default_rng(70 + kind)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    lx, lz = 12e-6, 7e-6
    o = np.array([1e-4, -2e-4, 3e-4])
    b = GeometryBuilder()
    (b.rect if kind == 0 else b.right_tri)(o, lx * q[:, 0], lz * q[:, 1])
    g = b.build("one", Images(), o - 1, o + 1)
    D = math.hypot(lx, lz)
    c = o + (0.5 if kind == 0 else 1 / 3) * (lx * q[:, 0] + lz * q[:, 1])
    d = rng.standard_normal((4000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    R = D * 10 ** rng.uniform(-2, 3, 4000)
    pts = c + R[:, None] * d
    dp = nb.DevicePanels.from_geometry(g, DEV)
    got = stack(nb.eval_points(dp, dev(np.ones(1)), *cols(pts), precision=nb.MIXED))
    ref = oracle.eval_points(g, np.ones(1), pts)
    ep = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
    eE = np.linalg.norm(got[:, 1:] - ref[:, 1:], axis=1) / np.linalg.norm(ref[:, 1:], axis=1)
    near = R < 4 * D
    assert ep[near].max() < 1e-10 and eE[near].max() < 1e-10
    assert ep[~near].max() < 5e-7 and eE[~near].max() < 5e-7, (ep[~near].max(), eE[~near].max())


def test_mixed_eval_gem_sampled(nb):
    g = gem_cell()
    rng = np.random.default_rng(71)
    sigma = rng.normal(0, 1e-5, g.n)
    pts = gem_eval_points(g, 5000, seed=12)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    got = stack(nb.eval_points(dp, dev(sigma), *cols(pts), precision=nb.MIXED))
    idx = rng.choice(len(pts), 40, replace=False)
    ref = oracle.eval_points(g, sigma, pts[idx])
    ephi, eE = rel_errors(got[idx], ref)
    assert ephi < 1e-6 and eE < 1e-6, (ephi, eE)


def test_mixed_assembly_is_exact(nb, small_gem):
    """The matrix is assembled with the exact closed forms in both modes."""
    g, A_ref, _, _, _ = small_gem
    dp = nb.DevicePanels.from_geometry(g, DEV)
    A = nb.assemble(dp, precision=nb.MIXED).cpu().numpy().T
    assert np.array_equal(A, nb.assemble(dp, precision=nb.FP64).cpu().numpy().T)
    err = np.abs(A - A_ref) / np.abs(A_ref).max(axis=1, keepdims=True)
    assert err.max() < 1e-10, err.max()


def test_mixed_solve_refines_to_fp64(nb, small_gem):
    g, A_ref, s_ref, _, _ = small_gem
    At = dev(np.ascontiguousarray(A_ref.T))
    b = g.rhs()
    sigma, ipiv, info = nb.solve(At, dev(b), precision=nb.MIXED)
    s = sigma.cpu().numpy()
    assert 1 <= info.ir_iters <= 30 and info.rel_resid <= 1e-10
    # the matrix is untouched in mixed mode
    assert np.array_equal(At.cpu().numpy().T, A_ref)
    r = A_ref @ s - b
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    kappa = np.linalg.cond(A_ref, 1)
    assert np.abs(s - s_ref).max() <= kappa * 2e-10 * np.abs(s_ref).max()


def test_mixed_solve_refinement_error_paths(nb, small_gem):
    g, A_ref, _, _, _ = small_gem
    At = dev(np.ascontiguousarray(A_ref.T))
    with pytest.raises(nb.NebemError) as e:
        nb.solve(At, dev(g.rhs()), precision=nb.MIXED, ir_max_iter=0)
    assert e.value.code == nb.NEBEM_ENOCONV
    with pytest.raises(nb.NebemError) as e:
        nb.solve(At, dev(g.rhs()), precision=nb.MIXED, ir_tol=1e-30)
    assert e.value.code == nb.NEBEM_ENOCONV


# ------------------------------------------------------------------ sessions

@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_session_pipeline(nb, small_gem, precision, tol):
    """assemble -> factor -> solve -> evaluate inside a session, vs the oracle
    pipeline; then a new right-hand side on the resident factors."""
    g, A_ref, s_ref, pts, f_ref = small_gem
    dp = nb.DevicePanels.from_geometry(g, DEV)
    ses = nb.Session(dp, precision=precision)
    assert ses.create_status == nb.NEBEM_OK
    s = ses.sigma().cpu().numpy()
    if precision == nb.FP64:
        kappa = np.linalg.cond(A_ref, 1)
        assert np.abs(s - s_ref).max() <= 100 * kappa * 2.2e-16 * np.abs(s_ref).max()
    got = stack(ses.eval_points(*cols(pts)))
    ephi, eE = rel_errors(got, f_ref)
    assert ephi < tol and eE < tol, (ephi, eE)
    # weighting-field style re-solve: unit potential on the top copper only.
    # Two independent pipelines differ by the solve's forward error (c kappa u
    # relative in sigma); the weighting potential is small in much of the
    # gap, so the end-to-end bound scales with kappa_1(A).
    b = np.where((g.bc == 0) & (g.value == -200.0), 1.0, 0.0)
    code, info = ses.solve(dev(b))
    assert code == nb.NEBEM_OK
    ref_w = oracle.solve(A_ref, b)
    pw = stack(ses.eval_points(*cols(pts)))
    fw = oracle.eval_points(g, ref_w, pts)
    ephi, eE = rel_errors(pw, fw)
    kappa = np.linalg.cond(A_ref, 1)
    tol_w = max(tol, 10 * kappa * 2.2e-16)
    assert ephi < tol_w and eE < tol_w, (ephi, eE, kappa)
    ses.close()


# -------------------------------------------------------------- space charge

def _charges(g, n, seed):
    c = np.array([0.5 * (g.images.a1[0] + g.images.a2[0]), 0.5 * g.images.a2[1], 0.0])
    return charge_cloud(c, 20e-6, n, seed)


def test_spacecharge_step_matches_oracle(nb, small_gem):
    g, A_ref, s_ref, _, _ = small_gem
    xyz, q = _charges(g, 2048, 13)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    ses = nb.Session(dp, precision=nb.FP64)
    qx, qy, qz = cols(xyz)
    E = tuple(torch.empty(len(q), dtype=torch.float64, device=DEV) for _ in range(3))
    ses.spacecharge_step(qx, qy, qz, dev(q), 0, E=E)
    torch.cuda.synchronize()
    params = oracle.SpaceChargeParams()
    new_ref, sig_ref, E_ref = oracle.spacecharge_step(g, A_ref, g.rhs(), s_ref, xyz, q, 0, params)
    s = ses.sigma().cpu().numpy()
    # sigma of two independent FP64 solves agrees to about kappa x u: this
    # matrix has kappa_1 = 3.3e6, and perturbing its entries by 1e-16
    # relative already moves sigma by 4.5e-10 of its maximum
    kappa = np.linalg.cond(A_ref, 1)
    assert np.abs(s - sig_ref).max() <= max(1e-9, 10 * kappa * 2.2e-16) * np.abs(sig_ref).max()
    Eg = np.column_stack([t.cpu().numpy() for t in E])
    # condition-normalised error of the charge-charge part: bound by the sum of |pair terms|
    abs_terms = np.zeros(len(q))
    d = xyz[:, None, :] - xyz[None, :, :]
    r = np.linalg.norm(d, axis=2)
    np.fill_diagonal(r, np.inf)
    abs_terms = oracle.ke() * (np.abs(q)[None, :] / r**2).sum(axis=1)
    err = np.linalg.norm(Eg - E_ref, axis=1)
    assert np.max(err / (abs_terms + np.linalg.norm(E_ref, axis=1))) < 1e-6
    moved = np.column_stack([t.cpu().numpy() for t in (qx, qy, qz)])
    disp_ref = np.linalg.norm(new_ref - xyz, axis=1)
    assert np.max(np.linalg.norm(moved - new_ref, axis=1) / disp_ref) < 1e-5
    ses.close()


@pytest.mark.parametrize("placement", ["centre", "weighted"])
def test_spacecharge_step_lines_matches_oracle(nb, small_gem, placement):
    """The step with line charges (Algorithm 3) against the oracle's pieces:
    voxel lines, their potential / normal field at the collocation points
    on the right-hand side, the FP64 solve, the panel field plus the
    charges' own field (far voxels as lines, near voxels as point charges)
    at every charge, and the move."""
    g, A_ref, _, _, _ = small_gem
    xyz, q = _charges(g, 3000, 16)
    c0 = np.array([0.5 * (g.images.a1[0] + g.images.a2[0]), 0.5 * g.images.a2[1], 0.0])
    origin, step, shape = c0 - 60e-6, (10e-6,) * 3, (12,) * 3
    dp = nb.DevicePanels.from_geometry(g, DEV)
    ses = nb.Session(dp, precision=nb.FP64)
    qx, qy, qz = cols(xyz)
    E = tuple(torch.empty(len(q), dtype=torch.float64, device=DEV) for _ in range(3))
    code, nl = ses.spacecharge_step_lines(qx, qy, qz, dev(q), 0, origin, step, shape, E=E, placement=placement)
    torch.cuda.synchronize()
    assert code == nb.NEBEM_OK
    lines, _ = oracle.voxel_lines(xyz, q, origin, step, shape, placement=placement)
    assert nl == len(lines)
    f = oracle.line_field(lines, g.centroids())
    en = np.einsum("ij,ij->i", f[:, 1:], g.normals())
    b = np.where(g.bc == 0, g.rhs() - f[:, 0], -en)
    sig_ref = oracle.solve(A_ref, b)
    s = ses.sigma().cpu().numpy()
    kappa = np.linalg.cond(A_ref, 1)
    assert np.abs(s - sig_ref).max() <= max(1e-9, 10 * kappa * 2.2e-16) * np.abs(sig_ref).max()
    # E from the session's own sigma (checked against the oracle's solve
    # above), so that the comparison is of the field sums alone
    E_pan = oracle.eval_points(g, s, xyz)[:, 1:]
    E_q, S = oracle.charge_field_lines(xyz, q, origin, step, shape, placement)
    E_ref = E_pan + E_q
    Eg = np.column_stack([t.cpu().numpy() for t in E])
    assert np.isfinite(Eg).all() and np.isfinite(E_ref).all()
    # scale: the panel part's magnitude and the charges' terms' (FP32 pairs)
    scale = np.linalg.norm(E_pan, axis=1) + S
    err = np.linalg.norm(Eg - E_ref, axis=1) / scale
    assert np.max(err) < 1e-6, np.max(err)
    moved = np.column_stack([t.cpu().numpy() for t in (qx, qy, qz)])
    p = oracle.SpaceChargeParams()
    new_ref = xyz + (np.sign(q) * p.mobility * p.dt)[:, None] * E_ref
    dmax = (p.mobility * p.dt * scale)
    assert np.max(np.linalg.norm(moved - new_ref, axis=1) / dmax) < 1e-6
    ses.close()


def test_spacecharge_newton_third_law_and_resolve_schedule(nb, small_gem):
    """Charge-charge forces sum to zero; sigma is re-solved only on multiples
    of sc_resolve_every."""
    g = small_gem[0]
    xyz, q = _charges(g, 20000, 14)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    ses = nb.Session(dp, precision=nb.FP64, sc_resolve_every=3)
    qx, qy, qz = cols(xyz)
    qd = dev(q)
    E = tuple(torch.empty(len(q), dtype=torch.float64, device=DEV) for _ in range(3))
    s0 = ses.sigma().cpu().numpy()
    ses.spacecharge_step(qx, qy, qz, qd, 1, E=E)     # no re-solve at step 1
    assert np.array_equal(ses.sigma().cpu().numpy(), s0)
    # panel part at the start-of-step positions, to isolate the charge part
    p0 = cols(xyz)
    panel = stack(ses.eval_points(*p0))[:, 1:]
    Ec = np.column_stack([t.cpu().numpy() for t in E]) - panel
    f = (q[:, None] * Ec).sum(axis=0)
    scale = np.abs(q[:, None] * Ec).sum()
    assert np.abs(f).max() < 1e-6 * scale
    ses.spacecharge_step(qx, qy, qz, qd, 3, E=E)     # re-solve at step 3
    assert not np.array_equal(ses.sigma().cpu().numpy(), s0)
    ses.close()


def test_spacecharge_threshold_rule(nb, small_gem):
    """Algorithm 4's SpChTh: with sc_threshold >= 0 sigma is re-solved at a
    step exactly when the charges' magnitude sum |q| exceeds it."""
    g = small_gem[0]
    xyz, q = _charges(g, 3000, 17)
    qabs = np.abs(q).sum()
    dp = nb.DevicePanels.from_geometry(g, DEV)
    for thr, resolves in ((2.0 * qabs, False), (0.5 * qabs, True)):
        ses = nb.Session(dp, precision=nb.FP64, sc_threshold=thr)
        s0 = ses.sigma().cpu().numpy()
        qx, qy, qz = cols(xyz)
        for k in (0, 1):  # the schedule would re-solve at step 0 only; the rule at both or neither
            before = ses.sigma().cpu().numpy()
            ses.spacecharge_step(qx, qy, qz, dev(q), k)
            torch.cuda.synchronize()
            after = ses.sigma().cpu().numpy()
            assert (not np.array_equal(before, after)) == resolves, (thr, k)
        if not resolves:
            assert np.array_equal(ses.sigma().cpu().numpy(), s0)
        ses.close()


@pytest.mark.parametrize("lines", [False, True])
def test_spacecharge_fastvol_regenerated(nb, small_gem, lines):
    """Algorithm 4's CreateFastVolPF: a FastVolume map attached to the
    session holds the panels' field now, and after a re-solve the panels'
    field with the new sigma plus the charges' own field (point charges or
    their lines) at the start-of-step positions."""
    g = small_gem[0]
    xyz, q = _charges(g, 2000, 18)
    c0 = np.array([0.5 * (g.images.a1[0] + g.images.a2[0]), 0.5 * g.images.a2[1], 0.0])
    origin, step, shape = tuple(c0 + np.array([-60e-6, -60e-6, 40e-6])), (10e-6, 12e-6, 15e-6), (13, 11, 9)
    vox = (tuple(c0 - 60e-6), (10e-6,) * 3, (12,) * 3)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    ses = nb.Session(dp, precision=nb.FP64)
    vals = ses.fastvol(grid=(origin, step, shape))
    torch.cuda.synchronize()
    nodes = oracle.grid_nodes(origin, step, shape)
    direct = stack(ses.eval_points(*cols(nodes)))
    assert np.array_equal(vals.cpu().numpy(), direct)
    qx, qy, qz = cols(xyz)
    if lines:
        ses.spacecharge_step_lines(qx, qy, qz, dev(q), 0, *vox)
    else:
        ses.spacecharge_step(qx, qy, qz, dev(q), 0)
    torch.cuda.synchronize()
    got = vals.cpu().numpy()
    panels = stack(ses.eval_points(*cols(nodes)))  # the new sigma
    assert not np.array_equal(panels, direct)
    if lines:
        ln, _ = oracle.voxel_lines(xyz, q, *vox)
        ref = oracle.line_field(ln, nodes)
        tol = 1e-10
        scale = np.abs(ref).max(axis=0)
    else:
        ref, S = oracle.coulomb(nodes, xyz, q, with_abs=True)
        tol = 1e-6
        scale = np.column_stack([S * 0 + np.abs(ref[:, 0]).max(), S, S, S])
    charge_part = got - panels
    assert np.all(np.abs(charge_part - ref) <= tol * (scale + np.abs(panels).max(axis=0) * 1e-6)), \
        np.max(np.abs(charge_part - ref) / (scale + 1e-300))
    ses.fastvol()  # detach
    ses.spacecharge_step(qx, qy, qz, dev(q), 10 if not lines else 10)
    torch.cuda.synchronize()
    assert np.array_equal(vals.cpu().numpy(), got)
    ses.close()


def test_spacecharge_deterministic(nb, small_gem):
    g = small_gem[0]
    xyz, q = _charges(g, 5000, 15)
    out = []
    for _ in range(2):
        dp = nb.DevicePanels.from_geometry(g, DEV)
        ses = nb.Session(dp)
        qx, qy, qz = cols(xyz)
        for k in range(3):
            ses.spacecharge_step(qx, qy, qz, dev(q), k)
        torch.cuda.synchronize()
        out.append(np.column_stack([t.cpu().numpy() for t in (qx, qy, qz)]))
        ses.close()
    assert np.array_equal(out[0], out[1])


# ------------------------------------------- full-size run, sampled outputs

def test_gem_full_size_sampled(nb):
    """The benchmark's configuration (8064 elements, 121 copies, 10^6 points),
    FP64 and mixed, checked on 64 sampled points against the oracle with a
    seeded density."""
    g = gem_cell()
    rng = np.random.default_rng(72)
    sigma = rng.normal(0, 1e-5, g.n)
    pts = gem_eval_points(g, 1_000_000, seed=1)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    idx = rng.choice(len(pts), 64, replace=False)
    ref = oracle.eval_points(g, sigma, pts[idx])
    for prec, tol in ((nb.FP64, 1e-10), (nb.MIXED, 1e-6)):
        got = stack(nb.eval_points(dp, dev(sigma), *cols(pts), precision=prec))
        assert np.all(np.isfinite(got))
        ephi, eE = rel_errors(got[idx], ref)
        assert ephi < tol and eE < tol, (prec, ephi, eE)


def test_thgem_sampled(nb):
    """Double THGEM (41 600 elements, 121 copies): FP64 and mixed evaluation
    on 16 sampled points against the oracle with a seeded density."""
    from synth import thgem_double, thgem_eval_points
    g = thgem_double()
    rng = np.random.default_rng(73)
    sigma = rng.normal(0, 1e-5, g.n)
    pts = thgem_eval_points(g, 4096, seed=2)
    idx = rng.choice(len(pts), 16, replace=False)
    ref = oracle.eval_points(g, sigma, pts[idx])
    dp = nb.DevicePanels.from_geometry(g, DEV)
    for prec, tol in ((nb.FP64, 1e-10), (nb.MIXED, 1e-6)):
        got = stack(nb.eval_points(dp, dev(sigma), *cols(pts[idx]), precision=prec))
        ephi, eE = rel_errors(got, ref)
        assert ephi < tol and eE < tol, (prec, ephi, eE)
