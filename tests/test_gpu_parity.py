"""Parity of the HIP path (through the C-ABI) against the CPU oracle.

FP64 bar (stated in the path's requirements): 1e-10 relative on phi and E,
pointwise, on points where |phi_ref| >= 1e-3 max|phi_ref| (|E_ref| likewise);
single-element kernels are held to the same bound at every distance.
Matrices: entry-wise relative to the row's largest entry.  Solves: residual
and forward error bounded by the condition number.
"""
import math

import numpy as np
import pytest

import oracle
from synth import GeometryBuilder, Images, gem_cell, parallel_plates, uniform_points
from synth.geometry import CONDUCTOR, DIELECTRIC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nb():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2606_24154_amd as nb
    return nb


DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def gpu_eval(nb, geom, sigma, pts, **kw):
    dp = nb.DevicePanels.from_geometry(geom, DEV)
    out = nb.eval_points(dp, dev(sigma), dev(pts[:, 0]), dev(pts[:, 1]), dev(pts[:, 2]), **kw)
    torch.cuda.synchronize()
    return np.column_stack([t.cpu().numpy() for t in out])


def cols(pts):
    return [dev(pts[:, k]) for k in range(3)]


def stack(out):
    torch.cuda.synchronize()
    return np.column_stack([t.cpu().numpy() for t in out])


def rel_errors(got, ref, floor=1e-3):
    """max pointwise relative error of phi and |E| on non-negligible points"""
    ap = np.abs(ref[:, 0])
    sel = ap >= floor * ap.max()
    ephi = np.max(np.abs(got[sel, 0] - ref[sel, 0]) / ap[sel])
    en = np.linalg.norm(ref[:, 1:], axis=1)
    sel = en >= floor * en.max()
    eE = np.max(np.linalg.norm(got[sel, 1:] - ref[sel, 1:], axis=1) / en[sel])
    return ephi, eE


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))


# ------------------------------------------------------------ single panels

@pytest.mark.parametrize("kind", [0, 1])
def test_single_panel_all_distances(nb, kind):
    """Unit-density element vs the oracle at distances 1e-3 D .. 1e3 D,
    including points just above/below the plane inside and outside it."""
    rng = np.random.default_rng(40 + kind)
    worst = [0.0, 0.0]
    for trial in range(6):
        Q = _rot(rng)
        lx, lz = rng.uniform(2e-6, 40e-6, 2)
        o = rng.uniform(-1e-3, 1e-3, 3)
        u, w = lx * Q[:, 0], lz * Q[:, 1]
        b = GeometryBuilder()
        (b.rect if kind == 0 else b.right_tri)(o, u, w)
        g = b.build("one", Images(), o - 1, o + 1)
        D = math.hypot(lx, lz)
        c = o + (0.5 if kind == 0 else 1 / 3) * (u + w)
        m = 3000
        d = rng.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        R = D * 10 ** rng.uniform(-3, 3, m)
        pts = c + R[:, None] * d
        # near-plane points over and beside the element
        k = m // 5
        s, t = rng.uniform(-0.3, 1.3, (2, k))
        n = np.cross(u, w) / np.linalg.norm(np.cross(u, w))
        h = D * 10 ** rng.uniform(-6, -1, k) * rng.choice([-1, 1], k)
        pts[:k] = o + s[:, None] * u + t[:, None] * w + h[:, None] * n
        sigma = np.array([1.0])
        got = gpu_eval(nb, g, sigma, pts)
        ref = oracle.eval_points(g, sigma, pts)
        ephi = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
        eE = np.linalg.norm(got[:, 1:] - ref[:, 1:], axis=1) / np.linalg.norm(ref[:, 1:], axis=1)
        worst = [max(worst[0], ephi.max()), max(worst[1], eE.max())]
    assert worst[0] < 1e-10 and worst[1] < 1e-10, worst


@pytest.mark.parametrize("kind", [0, 1])
def test_far_regime_switch_and_element_plane(nb, kind):
    """Points around the switch between the general and the far-regime
    evaluation (distance from the corner o of 4.5 .. 6 diameters), and points
    in the element's plane 5 .. 50 diameters away (normal field 0 there),
    against the oracle at the FP64 bar."""
    rng = np.random.default_rng(60 + kind)
    for trial in range(4):
        Q = _rot(rng)
        lx, lz = rng.uniform(2e-6, 40e-6, 2)
        o = rng.uniform(-1e-3, 1e-3, 3)
        u, w = lx * Q[:, 0], lz * Q[:, 1]
        b = GeometryBuilder()
        (b.rect if kind == 0 else b.right_tri)(o, u, w)
        g = b.build("one", Images(), o - 1, o + 1)
        D = math.hypot(lx, lz)
        d = rng.standard_normal((2000, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        pts = o + (D * rng.uniform(4.5, 6.0, 2000))[:, None] * d
        ang = rng.uniform(0, 2 * np.pi, 500)
        r = D * rng.uniform(5.0, 50.0, 500)
        inplane = o + (r * np.cos(ang))[:, None] * Q[:, 0] + (r * np.sin(ang))[:, None] * Q[:, 1]
        pts = np.vstack([pts, inplane])
        sigma = np.array([1.0])
        got = gpu_eval(nb, g, sigma, pts)
        ref = oracle.eval_points(g, sigma, pts)
        ephi = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
        eE = np.linalg.norm(got[:, 1:] - ref[:, 1:], axis=1) / np.linalg.norm(ref[:, 1:], axis=1)
        assert ephi.max() < 1e-10 and eE.max() < 1e-10, (trial, ephi.max(), eE.max())
        # in-plane points: the field has no component along the normal
        n = np.cross(u, w) / np.linalg.norm(np.cross(u, w))
        en = np.abs(got[2000:, 1:] @ n) / np.linalg.norm(got[2000:, 1:], axis=1)
        assert en.max() < 1e-10, en.max()


def _pair_geometry(rng, n_tri, copies=0):
    """n_tri general triangles with random orientation, each cut by the
    builder into its two right triangles (consecutive elements sharing the
    right-angle corner and a leg), lattice copies +-copies"""
    b = GeometryBuilder()
    for _ in range(n_tri):
        Q = _rot(rng)
        c0 = rng.uniform(-100e-6, 100e-6, 3)
        p3 = [c0 + rng.uniform(5e-6, 30e-6) * (np.cos(t) * Q[:, 0] + np.sin(t) * Q[:, 1])
              for t in np.sort(rng.uniform(0, 2 * np.pi, 3))]
        b.triangle(*p3)
    img = Images(a1=np.array([400e-6, 0, 0]), a2=np.array([0, 400e-6, 0]), n1=copies, n2=copies)
    return b.build("pairs", img, np.full(3, -1e-3), np.full(3, 1e-3))


def test_triangle_pairs_against_oracle_and_singles(nb):
    """Right-triangle pairs (a triangle cut at its altitude's foot) are
    evaluated together; against the oracle at the FP64 bar at 1e-3 .. 1e3
    diameters and near the plane, and against the same triangles with every
    pair's halves apart in the element order (first halves, then second
    halves: never paired) to 1e-11."""
    rng = np.random.default_rng(77)
    g = _pair_geometry(rng, 24, copies=2)
    assert g.n == 48 and np.all(g.kind == 1)
    sigma = rng.uniform(0.5, 1.5, g.n) * rng.choice([-1, 1], g.n)
    m = 3000
    d = rng.standard_normal((m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = rng.uniform(-100e-6, 100e-6, 3) + (30e-6 * 10 ** rng.uniform(-2, 2.3, m))[:, None] * d
    got = gpu_eval(nb, g, sigma, pts)
    ref = oracle.eval_points(g, sigma, pts)
    ephi, eE = rel_errors(got, ref)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)
    # the same elements with each pair's halves apart: no pairs
    perm = np.concatenate([np.arange(0, g.n, 2), np.arange(1, g.n, 2)])
    gs = g.subset(perm)
    got_s = gpu_eval(nb, gs, sigma[perm], pts)
    ephi, eE = rel_errors(got, got_s)
    assert ephi < 1e-11 and eE < 1e-11, (ephi, eE)
    assert not np.array_equal(got, got_s)  # the pair path did run


def test_triangle_pairs_mixed_against_oracle_and_singles(nb):
    """The mixed path's triangle pairs (one multipole expansion per far pair
    copy, each triangle's own tiers nearer): against the oracle at the mixed
    bar, at distances reaching past 96 diameters of the whole triangles, and
    against the same triangles with every pair's halves apart (single-element
    tiers) at the same bar."""
    rng = np.random.default_rng(79)
    g = _pair_geometry(rng, 24, copies=3)
    sigma = rng.uniform(0.5, 1.5, g.n) * rng.choice([-1, 1], g.n)
    m = 4000
    d = rng.standard_normal((m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = (30e-6 * 10 ** rng.uniform(0, 2.5, m))[:, None] * d
    got = gpu_eval(nb, g, sigma, pts, precision=nb.MIXED)
    ref = oracle.eval_points(g, sigma, pts)
    ephi, eE = rel_errors(got, ref)
    assert ephi < 1e-6 and eE < 1e-6, (ephi, eE)
    perm = np.concatenate([np.arange(0, g.n, 2), np.arange(1, g.n, 2)])
    got_s = gpu_eval(nb, g.subset(perm), sigma[perm], pts, precision=nb.MIXED)
    ephi, eE = rel_errors(got, got_s)
    assert ephi < 1e-6 and eE < 1e-6, (ephi, eE)
    assert not np.array_equal(got, got_s)


def test_triangle_pair_at_tile_edge(nb):
    """A pair whose second triangle falls into the next tile of 64 elements
    is evaluated as two single triangles; every element still counted once."""
    rng = np.random.default_rng(78)
    b = GeometryBuilder()
    for k in range(63):  # 63 rectangles, then the pair at positions 63, 64
        b.rect(rng.uniform(-1e-4, 1e-4, 3), (10e-6, 0, 0), (0, 10e-6, 0))
    pg = _pair_geometry(rng, 2)
    g0 = b.build("edge", Images(), np.full(3, -1e-3), np.full(3, 1e-3))
    idx = np.arange(pg.n)
    g = type(g0)("edge", np.concatenate([g0.kind, pg.kind]), np.vstack([g0.o, pg.o]), np.vstack([g0.u, pg.u]),
                 np.vstack([g0.w, pg.w]), np.concatenate([g0.bc, pg.bc]), np.concatenate([g0.value, pg.value]),
                 np.concatenate([g0.eps_pos, pg.eps_pos]), np.concatenate([g0.eps_neg, pg.eps_neg]), Images(),
                 g0.box_lo, g0.box_hi)
    assert g.n == 63 + len(idx)
    sigma = rng.uniform(0.5, 1.5, g.n)
    pts = uniform_points(np.full(3, -3e-4), np.full(3, 3e-4), 512, 5)
    got = gpu_eval(nb, g, sigma, pts)
    ref = oracle.eval_points(g, sigma, pts)
    ephi, eE = rel_errors(got, ref)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)


# -------------------------------------------------------- parallel plates

@pytest.fixture(scope="module")
def plates_ref():
    g = parallel_plates()
    A = oracle.assemble(g)
    s = oracle.solve(A, g.rhs())
    pts = uniform_points(g.box_lo, g.box_hi, 4096, 0)
    f = oracle.eval_points(g, s, pts)
    return g, A, s, pts, f


def test_plates_assembly(nb, plates_ref):
    g, A_ref, _, _, _ = plates_ref
    dp = nb.DevicePanels.from_geometry(g, DEV)
    At = nb.assemble(dp)
    torch.cuda.synchronize()
    A = At.cpu().numpy().T
    err = np.abs(A - A_ref) / np.abs(A_ref).max(axis=1, keepdims=True)
    assert err.max() < 1e-12, err.max()


def test_plates_solve_and_eval(nb, plates_ref):
    g, A_ref, s_ref, pts, f_ref = plates_ref
    At = dev(np.ascontiguousarray(A_ref.T))  # column-major storage
    b = dev(g.rhs())
    sigma, ipiv, info = nb.solve(At, b)
    torch.cuda.synchronize()
    s = sigma.cpu().numpy()
    kappa = np.linalg.cond(A_ref, 1)
    assert np.abs(s - s_ref).max() <= 50 * kappa * 2.2e-16 * np.abs(s_ref).max()
    got = gpu_eval(nb, g, s_ref, pts)
    ephi, eE = rel_errors(got, f_ref)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)


def test_fp64_solve_refinement(nb):
    """FP64 solve = LU + FP64 refinement: the returned x has no larger
    residual than the LU solution (re-solved from the returned factors), its
    error against the known solution is no larger, and info reports the true
    residual of the returned x."""
    rng = np.random.default_rng(11)
    n = 700
    qa, _ = np.linalg.qr(rng.standard_normal((n, n)))
    qb, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (qa * np.logspace(0, -9, n)) @ qb.T  # cond 1e9
    x_true = rng.standard_normal(n)
    b = A @ x_true
    At = dev(np.ascontiguousarray(A.T))
    sigma, ipiv, info = nb.solve(At, dev(b))
    x_lu = nb.solve_factored(At, ipiv, dev(b))
    torch.cuda.synchronize()
    x, xl = sigma.cpu().numpy(), x_lu.cpu().numpy()
    res = lambda v: np.linalg.norm(b - A @ v) / np.linalg.norm(b)
    # residuals near the FP64 floor: GPU and CPU evaluations of b - A x differ
    # by their own rounding, so the comparisons allow a factor 2
    assert 0 <= info.ir_iters <= 3
    assert res(x) <= 2 * res(xl), (res(x), res(xl))
    assert 0 < info.rel_resid < 1e-12 and res(x) < 1e-12, (info.rel_resid, res(x))
    assert np.linalg.norm(x - x_true) <= 1.5 * np.linalg.norm(xl - x_true)


def test_plates_end_to_end(nb, plates_ref):
    """assemble -> solve -> eval entirely on the GPU vs the oracle pipeline."""
    g, _, s_ref, pts, f_ref = plates_ref
    dp = nb.DevicePanels.from_geometry(g, DEV)
    At = nb.assemble(dp)
    sigma, _, _ = nb.solve(At, dev(g.rhs()))
    out = nb.eval_points(dp, sigma, dev(pts[:, 0]), dev(pts[:, 1]), dev(pts[:, 2]))
    torch.cuda.synchronize()
    got = np.column_stack([t.cpu().numpy() for t in out])
    ephi, eE = rel_errors(got, f_ref)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)


# ------------------------------------------------------ weighting fields

@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_eval_multi_equals_single_columns(nb, prec):
    """Several density columns in one evaluation: column k equals the
    single-column evaluation bit for bit, on the unordered (m < 4096) and
    Morton-ordered paths, with 6 columns (a chunk of 4 and one of 2)."""
    P = nb.FP64 if prec == "fp64" else nb.MIXED
    rng = np.random.default_rng(31)
    g = _mixed_geometry(rng, n=20).with_images(
        Images(a1=np.array([1.5e-3, 0, 0]), a2=np.array([0, 1.5e-3, 0]), n1=2, n2=1))
    dp = nb.DevicePanels.from_geometry(g, DEV)
    nsig = 6
    sig = rng.standard_normal((nsig, g.n)) * 1e-9
    for m in (1000, 5000):
        pts = uniform_points(g.box_lo, g.box_hi, m, m)
        pt = [dev(pts[:, k]) for k in range(3)]
        multi = nb.eval_points_multi(dp, dev(sig), *pt, precision=P)
        for k in range(nsig):
            single = nb.eval_points(dp, dev(sig[k]), *pt, precision=P)
            torch.cuda.synchronize()
            for c in range(4):
                assert torch.equal(multi[c][k], single[c]), (m, k, c)


def test_weighting_fields_plates(nb, plates_ref):
    """Weighting fields of the two plates (each at 1 V with the other at 0):
    multi-RHS solve, then both columns in one evaluation, against the
    oracle's solve and evaluation of each column; their sum is the field of
    both plates at 1 V."""
    g, A_ref, _, pts, _ = plates_ref
    top = (np.asarray(g.value) == 1.0).astype(float)
    B = np.stack([top, 1.0 - top])
    dp = nb.DevicePanels.from_geometry(g, DEV)
    At = nb.assemble(dp)
    sigma, _, _ = nb.solve(At, dev(B))
    out = nb.eval_points_multi(dp, sigma, dev(pts[:, 0]), dev(pts[:, 1]), dev(pts[:, 2]))
    torch.cuda.synchronize()
    got = [np.column_stack([t[k].cpu().numpy() for t in out]) for k in range(2)]
    for k in range(2):
        s_ref = oracle.solve(A_ref, B[k])
        f_ref = oracle.eval_points(g, s_ref, pts)
        ephi, eE = rel_errors(got[k], f_ref)
        assert ephi < 1e-10 and eE < 1e-10, (k, ephi, eE)
    both = oracle.eval_points(g, oracle.solve(A_ref, B[0] + B[1]), pts)
    ephi, eE = rel_errors(got[0] + got[1], both)
    # with both plates at 1 V the two columns' fields nearly cancel between
    # the plates, so E of the sum is small against either column's and its
    # relative error is the columns' (each < 1e-10) times that ratio
    assert ephi < 1e-10 and eE < 1e-9, (ephi, eE)


# ------------------------------------------------------------ FastVolume

FV_ORIGIN, FV_STEP, FV_SHAPE = (-0.3e-3, -0.25e-3, -0.04e-3), (1e-5, 1e-5, 1e-5), (61, 51, 9)


def test_fastvol_interp_matches_oracle(nb):
    """Trilinear lookup of arbitrary node values against the oracle's
    definition, inside, on the last nodes and outside (NaN)."""
    rng = np.random.default_rng(41)
    nn = int(np.prod(FV_SHAPE))
    vals = rng.standard_normal((nn, 4))
    lo = np.array(FV_ORIGIN)
    hi = lo + (np.array(FV_SHAPE) - 1) * np.array(FV_STEP)
    pts = rng.uniform(lo - 0.05 * (hi - lo), hi + 0.05 * (hi - lo), (3000, 3))
    pts[:20] = oracle.grid_nodes(FV_ORIGIN, FV_STEP, FV_SHAPE)[-20:]
    out = nb.fastvol_interp(dev(vals), FV_ORIGIN, FV_STEP, FV_SHAPE, *(dev(pts[:, k]) for k in range(3)))
    torch.cuda.synchronize()
    got = np.column_stack([t.cpu().numpy() for t in out])
    ref = oracle.trilinear(FV_ORIGIN, FV_STEP, FV_SHAPE, vals, pts)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert ok.sum() > 2000 and (~ok).sum() > 100
    assert np.abs(got[ok] - ref[ok]).max() <= 1e-14 * np.abs(vals).max()


def test_fastvol_build_and_error_vs_direct(nb, plates_ref):
    """Node values equal nebem_eval at the nodes bit for bit; between the
    plates the interpolated field stays within the paper's 0.25 % of the
    direct evaluation."""
    g, _, s_ref, _, _ = plates_ref
    dp = nb.DevicePanels.from_geometry(g, DEV)
    sig = dev(s_ref)
    vals = nb.fastvol_build(dp, sig, FV_ORIGIN, FV_STEP, FV_SHAPE)
    nodes = oracle.grid_nodes(FV_ORIGIN, FV_STEP, FV_SHAPE)
    direct = nb.eval_points(dp, sig, *(dev(nodes[:, k]) for k in range(3)))
    torch.cuda.synchronize()
    assert np.array_equal(vals.cpu().numpy(), np.column_stack([t.cpu().numpy() for t in direct]))
    rng = np.random.default_rng(42)
    lo = np.array(FV_ORIGIN)
    hi = lo + (np.array(FV_SHAPE) - 1) * np.array(FV_STEP)
    pts = rng.uniform(lo, hi, (4000, 3))
    pt = [dev(pts[:, k]) for k in range(3)]
    fi = np.column_stack([t.cpu().numpy() for t in nb.fastvol_interp(vals, FV_ORIGIN, FV_STEP, FV_SHAPE, *pt)])
    fd = np.column_stack([t.cpu().numpy() for t in nb.eval_points(dp, sig, *pt)])
    ephi = np.abs(fi[:, 0] - fd[:, 0]).max() / np.abs(fd[:, 0]).max()
    eE = (np.linalg.norm(fi[:, 1:] - fd[:, 1:], axis=1) / np.linalg.norm(fd[:, 1:], axis=1)).max()
    assert ephi < 2.5e-3 and eE < 2.5e-3, (ephi, eE)


FV_AXES = (np.array([-0.5e-3, -0.3e-3, -0.2e-3, -0.15e-3, -0.12e-3, 0.0, 0.1e-3, 0.35e-3, 0.5e-3]),
           np.array([-0.5e-3, -0.45e-3, -0.1e-3, 0.2e-3, 0.22e-3, 0.5e-3]),
           np.array([-0.09e-3, -0.085e-3, -0.07e-3, -0.03e-3, 0.02e-3, 0.06e-3, 0.08e-3, 0.089e-3]))


def test_fastvol_axes_interp_matches_oracle(nb):
    """Trilinear lookup on a graded grid (uneven node spacing per axis) of
    arbitrary node values against the oracle's definition, inside, on the
    last nodes, exactly on inner nodes and outside (NaN)."""
    rng = np.random.default_rng(43)
    nn = int(np.prod([len(a) for a in FV_AXES]))
    vals = rng.standard_normal((nn, 4))
    lo = np.array([a[0] for a in FV_AXES])
    hi = np.array([a[-1] for a in FV_AXES])
    pts = rng.uniform(lo - 0.05 * (hi - lo), hi + 0.05 * (hi - lo), (3000, 3))
    nodes = oracle.axes_nodes(FV_AXES)
    pts[:20] = nodes[-20:]
    pts[20:60] = nodes[rng.choice(nn, 40, replace=False)]
    ax = [dev(a) for a in FV_AXES]
    out = nb.fastvol_interp_axes(dev(vals), *ax, *(dev(pts[:, k]) for k in range(3)))
    torch.cuda.synchronize()
    got = np.column_stack([t.cpu().numpy() for t in out])
    ref = oracle.trilinear_axes(FV_AXES, vals, pts)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert ok.sum() > 2000 and (~ok).sum() > 100
    assert np.abs(got[ok] - ref[ok]).max() <= 1e-14 * np.abs(vals).max()


def test_fastvol_axes_build_and_validation(nb, plates_ref):
    """Graded-grid node values equal nebem_eval at the nodes bit for bit; an
    axis that is not strictly increasing is refused."""
    g, _, s_ref, _, _ = plates_ref
    dp = nb.DevicePanels.from_geometry(g, DEV)
    sig = dev(s_ref)
    ax = [dev(a) for a in FV_AXES]
    vals = nb.fastvol_build_axes(dp, sig, *ax)
    nodes = oracle.axes_nodes(FV_AXES)
    direct = nb.eval_points(dp, sig, *(dev(nodes[:, k]) for k in range(3)))
    torch.cuda.synchronize()
    assert np.array_equal(vals.cpu().numpy(), np.column_stack([t.cpu().numpy() for t in direct]))
    bad = FV_AXES[2].copy()
    bad[3] = bad[2]
    with pytest.raises(nb.NebemError) as e:
        nb.fastvol_build_axes(dp, sig, ax[0], ax[1], dev(bad))
    assert e.value.code == nb.NEBEM_EINVAL


# ------------------------------------------------ point -> line charges

@pytest.mark.parametrize("placement", ["centre", "weighted"])
def test_voxel_lines_match_oracle(nb, placement):
    """Algorithm 3's reduction against the oracle: same occupied voxels in
    the same order, same line placement and densities, same dropped count."""
    rng = np.random.default_rng(71)
    n = 20000
    xyz = rng.normal(0, 12e-6, (n, 3))
    q = np.where(np.arange(n) % 2, 1.0, -1.0) * 1.602176634e-19
    q[::7] *= 3.0
    origin, step, shape = (-30e-6, -30e-6, -30e-6), (5e-6, 4e-6, 5e-6), (12, 15, 12)
    lines, out = nb.voxelize_charges(*(dev(xyz[:, k]) for k in range(3)), dev(q), origin, step, shape,
                                     placement=placement)
    ref, ref_out = oracle.voxel_lines(xyz, q, origin, step, shape, placement=placement)
    got = lines.cpu().numpy()
    assert out == ref_out and out > 0
    assert got.shape == ref.shape
    np.testing.assert_allclose(got[:, :6], ref[:, :6], rtol=1e-13, atol=1e-12 * 60e-6)  # z = 0 rounds either way
    np.testing.assert_allclose(got[:, 6], ref[:, 6], rtol=0, atol=1e-12 * np.abs(ref[:, 6]).max())


@pytest.mark.parametrize("placement", ["centre", "weighted"])
def test_charge_field_lines_matches_oracle(nb, placement):
    """The charges' own field with far voxels as lines and the 27 voxels
    around each charge as point charges, against the oracle's definition;
    FP32 pair terms with FP64 sums: error bound 1e-6 of the sum of the
    terms' magnitudes.  Some charges outside the grid."""
    rng = np.random.default_rng(77)
    n = 3000
    xyz = rng.normal(0, 15e-6, (n, 3))
    q = np.where(np.arange(n) % 2, 1.0, -1.0) * 1.602176634e-19 * rng.uniform(0.5, 2.0, n)
    origin, step, shape = (-40e-6, -36e-6, -40e-6), (5e-6, 6e-6, 5e-6), (16, 12, 16)
    E, nl = nb.charge_field_lines(*(dev(xyz[:, k]) for k in range(3)), dev(q), origin, step, shape,
                                  placement=placement)
    torch.cuda.synchronize()
    ref, S = oracle.charge_field_lines(xyz, q, origin, step, shape, placement)
    lines, nout = oracle.voxel_lines(xyz, q, origin, step, shape, placement)
    assert nl == len(lines) and nout > 0
    got = np.column_stack([t.cpu().numpy() for t in E])
    assert np.isfinite(got).all()
    err = np.linalg.norm(got - ref, axis=1) / S
    assert err.max() < 1e-6, err.max()


def test_lone_charge_line_passes_through_it(nb):
    """A charge alone in its voxel gets a line through its own x, y exactly,
    and its field there across the line is the principal value 0."""
    rng = np.random.default_rng(74)
    ijk = rng.choice(10 ** 3, 200, replace=False)
    cell = np.column_stack([ijk % 10, (ijk // 10) % 10, ijk // 100]).astype(float)
    xyz = (cell + rng.uniform(0.05, 0.95, (200, 3))) * 7e-6 - 35e-6
    q = rng.choice([-1.0, 1.0], 200) * 1.602176634e-19 * rng.uniform(0.5, 3.0, 200)
    pts = [dev(np.ascontiguousarray(xyz[:, k])) for k in range(3)]
    lines, out = nb.voxelize_charges(*pts, dev(q), (-35e-6,) * 3, (7e-6,) * 3, (10,) * 3, placement="weighted")
    torch.cuda.synchronize()
    ln = lines.cpu().numpy()
    assert out == 0 and len(ln) == 200
    order = np.argsort(ijk)  # lines come in voxel order
    assert np.array_equal(ln[:, 0], xyz[order, 0]) and np.array_equal(ln[:, 1], xyz[order, 1])
    assert np.array_equal(ln[:, 3], xyz[order, 0]) and np.array_equal(ln[:, 4], xyz[order, 1])
    f = nb.line_field(lines[:1], *(t[order[:1]] for t in pts))
    torch.cuda.synchronize()
    assert f[1].item() == 0.0 and f[2].item() == 0.0 and np.isinf(f[0].item())


def test_line_field_matches_oracle(nb):
    """Segment field against the oracle's closed form, at points around,
    alongside and beyond the ends of the segments."""
    rng = np.random.default_rng(72)
    a = rng.uniform(-20e-6, 20e-6, (40, 3))
    b = a + rng.normal(0, 5e-6, (40, 3))
    lines = np.column_stack([a, b, rng.normal(0, 1e-12, 40)])
    pts = rng.uniform(-40e-6, 40e-6, (3000, 3))
    out = nb.line_field(dev(lines), *(dev(pts[:, k]) for k in range(3)))
    torch.cuda.synchronize()
    got = np.column_stack([t.cpu().numpy() for t in out])
    ref = oracle.line_field(lines, pts)
    ephi, eE = rel_errors(got, ref)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)


def test_line_field_single_segment_regimes(nb):
    """One segment, pointwise against the oracle: far away (10 to 10^4
    lengths), near the axis beyond either end, level with an end, and close
    beside it -- the places where the plain forms cancel."""
    rng = np.random.default_rng(73)
    a = np.array([1e-6, -2e-6, 3e-6])
    t = rng.normal(size=3)
    t /= np.linalg.norm(t)
    L = 5e-6
    b = a + L * t
    perp = np.cross(t, [0.3, 0.5, 0.8])
    perp /= np.linalg.norm(perp)
    mid = 0.5 * (a + b)
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    far = mid + d * (L * 10 ** rng.uniform(1, 4, (400, 1)))
    k = L * 10 ** rng.uniform(-1, 1, (200, 1))
    axis_a = a - k * t + 1e-3 * L * perp
    axis_b = b + k * t - 1e-3 * L * perp
    level = a + L * 10 ** rng.uniform(-2, 1, (200, 1)) * perp
    beside = a + rng.uniform(0.05, 0.95, (200, 1)) * L * t + L * 10 ** rng.uniform(-3, 0, (200, 1)) * perp
    pts = np.concatenate([far, axis_a, axis_b, level, beside])
    lines = np.concatenate([a, b, [3e-12]])[None, :]
    out = nb.line_field(dev(lines), *(dev(pts[:, k]) for k in range(3)))
    torch.cuda.synchronize()
    got = np.column_stack([t.cpu().numpy() for t in out])
    ref = oracle.line_field(lines, pts)
    ephi, eE = rel_errors(got, ref, floor=0.0)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)


# --------------------------------------------------- Adaptive Modelling

def test_adaptive_matches_oracle(nb):
    """Adaptive Modelling against the oracle's definition for PrimAfter -1
    .. 3 on the strip cell (copies +-3), with a reflection; PrimAfter >= 3
    (no far copies) equals nebem_eval bit for bit."""
    from synth import strip_cell
    e, p, emap = strip_cell(n_img=3, sub_u=2, sub_w=8)
    im = Images(a1=e.images.a1, a2=e.images.a2, n1=3, n2=3, mirror_mask=4,
                mirror_pos=np.array([0.0, 0.0, -60e-6]), mirror_parity=np.array([1, 1, -1], dtype=np.int32))
    e, p = e.with_images(im), p.with_images(im)
    rng = np.random.default_rng(61)
    sigma = (1.0 + 0.5 * rng.standard_normal(e.n)) * 1e-9
    pts = uniform_points(e.box_lo, e.box_hi, 1500, 61)
    dp, dpp = nb.DevicePanels.from_geometry(e, DEV), nb.DevicePanels.from_geometry(p, DEV)
    demap = torch.from_numpy(emap).to(DEV)
    pt = [dev(pts[:, k]) for k in range(3)]
    exact = nb.eval_points(dp, dev(sigma), *pt)
    for k in (-1, 0, 1, 2, 3):
        out = nb.eval_points_adaptive(dp, dpp, demap, k, dev(sigma), *pt)
        torch.cuda.synchronize()
        got = np.column_stack([t.cpu().numpy() for t in out])
        ref = oracle.eval_adaptive(e, p, emap, k, sigma, pts)
        ephi, eE = rel_errors(got, ref)
        assert ephi < 1e-10 and eE < 1e-10, (k, ephi, eE)
        if k < 0 or k >= 3:
            for c in range(4):
                assert torch.equal(out[c], exact[c]), (k, c)


def test_adaptive_rejects_bad_primitive_map(nb):
    """An element mapped to a primitive index outside [0, np) is refused
    (the map is checked on the device while the densities are summed)."""
    from synth import strip_cell
    e, p, emap = strip_cell(n_img=2, sub_u=2, sub_w=4)
    sigma = np.full(e.n, 1e-9)
    pts = uniform_points(e.box_lo, e.box_hi, 64, 62)
    dp, dpp = nb.DevicePanels.from_geometry(e, DEV), nb.DevicePanels.from_geometry(p, DEV)
    pt = [dev(pts[:, k]) for k in range(3)]
    for bad in (p.n, -1):
        m = emap.copy()
        m[e.n // 2] = bad
        with pytest.raises(nb.NebemError) as err:
            nb.eval_points_adaptive(dp, dpp, torch.from_numpy(m).to(DEV), 0, dev(sigma), *pt)
        assert err.value.code == nb.NEBEM_EINVAL


# ---------------------------------------------------- copies and mirrors

def _mixed_geometry(rng, n=24, bc_mix=True):
    b = GeometryBuilder()
    for i in range(n):
        Q = _rot(rng)
        o = rng.uniform(-0.4e-3, 0.4e-3, 3)
        lx, lz = rng.uniform(10e-6, 60e-6, 2)
        kw = dict(bc=CONDUCTOR, value=float(rng.uniform(-100, 100)))
        if bc_mix and i % 3 == 2:
            kw = dict(bc=DIELECTRIC, eps_pos=1.0, eps_neg=float(rng.uniform(2, 5)))
        (b.rect if i % 2 else b.right_tri)(o, lx * Q[:, 0], lz * Q[:, 1], **kw)
    return b.build("mixed", Images(), (-1e-3,) * 3, (1e-3,) * 3)


def test_lattice_and_mirror_copies(nb):
    rng = np.random.default_rng(50)
    g = _mixed_geometry(rng)
    sigma = rng.uniform(-1e-6, 1e-6, g.n)
    pts = uniform_points((-0.6e-3,) * 3, (0.6e-3,) * 3, 777, 51)
    for im in (Images(a1=np.array([1e-3, 0, 0]), a2=np.array([0.3e-3, 0.9e-3, 0.0]), n1=3, n2=2),
               Images(mirror_mask=5, mirror_pos=np.array([0.7e-3, 0, -0.6e-3]),
                      mirror_parity=np.array([-1, 1, 1], dtype=np.int32)),
               Images(a1=np.array([1.1e-3, 0, 0]), a2=np.array([0, 1.2e-3, 0]), n1=2, n2=1, mirror_mask=4,
                      mirror_pos=np.array([0, 0, -0.8e-3]), mirror_parity=np.array([1, 1, -1], dtype=np.int32))):
        gi = g.with_images(im)
        got = gpu_eval(nb, gi, sigma, pts)
        ref = oracle.eval_points(gi, sigma, pts)
        ephi, eE = rel_errors(got, ref)
        assert ephi < 1e-10 and eE < 1e-10, (im, ephi, eE)


def test_assembly_with_dielectric_rows_and_copies(nb):
    rng = np.random.default_rng(52)
    g = _mixed_geometry(rng, n=40).with_images(
        Images(a1=np.array([1e-3, 0, 0]), a2=np.array([0.5e-3, 0.85e-3, 0]), n1=2, n2=2))
    dp = nb.DevicePanels.from_geometry(g, DEV)
    A = nb.assemble(dp).cpu().numpy().T
    A_ref = oracle.assemble(g)
    err = np.abs(A - A_ref) / np.abs(A_ref).max(axis=1, keepdims=True)
    assert err.max() < 1e-11, err.max()


# ------------------------------------------------------------ GEM geometry

@pytest.fixture(scope="module")
def gem():
    return gem_cell()


def test_gem_assembly_sampled_rows(nb, gem):
    """Full 8064 x 8064 assembly with 121 copies on the GPU; 12 sampled rows
    (conductor and dielectric) against the oracle."""
    g = gem
    dp = nb.DevicePanels.from_geometry(g, DEV)
    At = nb.assemble(dp)
    torch.cuda.synchronize()
    rng = np.random.default_rng(53)
    rows = np.concatenate([rng.choice(np.where(g.bc == 0)[0], 6, replace=False),
                           rng.choice(np.where(g.bc == 1)[0], 6, replace=False), [0, g.n - 1]])
    ref = oracle.assemble_rows(g, rows)
    got = At[:, torch.from_numpy(rows).to(DEV)].cpu().numpy().T
    err = np.abs(got - ref) / np.abs(ref).max(axis=1, keepdims=True)
    assert err.max() < 1e-11, err.max()
    # backward error of the GPU solve on the GPU-assembled matrix
    A64 = At.cpu().numpy().T.copy()
    b = dev(g.rhs())
    sigma, _, _ = nb.solve(At, b)
    s = sigma.cpu().numpy()
    r = A64 @ s - g.rhs()
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(A64, 1) * np.linalg.norm(s)


def test_gem_eval_sampled_points(nb, gem):
    g = gem
    rng = np.random.default_rng(54)
    sigma = rng.normal(0, 1e-5, g.n)
    from synth import gem_eval_points
    pts = gem_eval_points(g, 2000, seed=1)
    got = gpu_eval(nb, g, sigma, pts)
    idx = rng.choice(len(pts), 48, replace=False)
    ref = oracle.eval_points(g, sigma, pts[idx])
    ephi, eE = rel_errors(got[idx], ref)
    assert ephi < 1e-10 and eE < 1e-10, (ephi, eE)


# ------------------------------------------------------------------- solve

@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 257, 777, 1029])
def test_lu_random(nb, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + np.eye(n) * 0.5
    B = rng.standard_normal((3, n))
    At = dev(np.ascontiguousarray(A.T))
    X, ipiv, info = nb.solve(At, dev(B))
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    ref = np.linalg.solve(A, B.T).T
    kappa = np.linalg.cond(A, 1)
    assert np.abs(X - ref).max() <= 100 * kappa * 2.2e-16 * max(1.0, np.abs(ref).max())
    # factors reproduce P A = L U
    LU = At.cpu().numpy().T
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    piv = ipiv.cpu().numpy()
    PA = A.copy()
    for k in range(n):
        PA[[k, piv[k]]] = PA[[piv[k], k]]
    assert np.abs(L @ U - PA).max() <= 1e-13 * n * np.abs(A).max()
    # partial pivoting: every multiplier bounded by 1
    assert np.abs(np.tril(LU, -1)).max() <= 1.0
    # re-solve from the resident factors (LU only; nb.solve also refined in
    # FP64, so the two agree to the solve's accuracy), deterministic
    X2 = nb.solve_factored(At, ipiv, dev(B)).cpu().numpy()
    assert np.abs(X2 - ref).max() <= 100 * kappa * 2.2e-16 * max(1.0, np.abs(ref).max())
    X3 = nb.solve_factored(At, ipiv, dev(B)).cpu().numpy()
    assert np.array_equal(X2, X3)


@pytest.mark.parametrize("n", [65, 777])
def test_lu_per_column_panels(nb, n, monkeypatch):
    """The per-column panel launches (taken when a panel's workgroups do not
    fit on the device at once) give the same factors as the single-launch
    panels: same pivots, and L U = P A."""
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n)) + np.eye(n) * 0.5
    b = rng.standard_normal(n)
    At1 = dev(np.ascontiguousarray(A.T))
    _, piv1, _ = nb.solve(At1, dev(b))
    monkeypatch.setenv("NEBEM_PANEL_PER_COLUMN", "1")
    At2 = dev(np.ascontiguousarray(A.T))
    _, piv2, _ = nb.solve(At2, dev(b))
    monkeypatch.delenv("NEBEM_PANEL_PER_COLUMN")
    torch.cuda.synchronize()
    assert np.array_equal(piv1.cpu().numpy(), piv2.cpu().numpy())
    LU1, LU2 = At1.cpu().numpy().T, At2.cpu().numpy().T
    assert np.abs(LU1 - LU2).max() <= 1e-12 * np.abs(LU1).max()
    L = np.tril(LU2, -1) + np.eye(n)
    U = np.triu(LU2)
    PA = A.copy()
    for k, p in enumerate(piv2.cpu().numpy()):
        PA[[k, p]] = PA[[p, k]]
    assert np.abs(L @ U - PA).max() <= 1e-13 * n * np.abs(A).max()


def test_condest_exact_case_and_random(nb):
    """cond_1 estimate: exact where the estimator's transposed step must
    find the one large column of A^-1 (A = I - M e_i e_j^T, A^-1 =
    I + M e_i e_j^T, i > j so that pivoting swaps rows), and a lower bound
    within a factor 10 on random matrices with known cond_1."""
    n, M, i0, j0 = 300, 1e6, 250, 40
    A = np.eye(n)
    A[i0, j0] = -M
    At = dev(np.ascontiguousarray(A.T))
    anorm = nb.norm1(At)
    assert anorm == 1.0 + M
    _, ipiv, _ = nb.solve(At, dev(np.ones(n)))
    est = nb.condest(At, ipiv, anorm)
    assert abs(est - (1 + M) ** 2) <= 1e-9 * (1 + M) ** 2, est
    rng = np.random.default_rng(21)
    for n in (70, 333):
        qa, _ = np.linalg.qr(rng.standard_normal((n, n)))
        qb, _ = np.linalg.qr(rng.standard_normal((n, n)))
        A = (qa * np.logspace(0, -6, n)) @ qb.T
        kappa = np.linalg.cond(A, 1)
        At = dev(np.ascontiguousarray(A.T))
        anorm = nb.norm1(At)
        assert abs(anorm - np.abs(A).sum(axis=0).max()) <= 1e-12 * anorm
        _, ipiv, _ = nb.solve(At, dev(np.ones(n)))
        est = nb.condest(At, ipiv, anorm)
        assert kappa / 10 <= est <= kappa * (1 + 1e-9), (est, kappa)


def test_session_condest(nb, plates_ref):
    g, A_ref, _, _, _ = plates_ref
    ses = nb.Session(nb.DevicePanels.from_geometry(g, DEV), precision=nb.FP64)
    est = ses.condest()
    kappa = np.linalg.cond(A_ref, 1)
    assert kappa / 10 <= est <= kappa * (1 + 1e-6), (est, kappa)
    ses.close()
    mixed = nb.Session(nb.DevicePanels.from_geometry(g, DEV), precision=nb.MIXED)
    with pytest.raises(nb.NebemError) as e:
        mixed.condest()
    assert e.value.code == nb.NEBEM_EINVAL
    mixed.close()


def test_lu_singular(nb):
    n = 70
    rng = np.random.default_rng(3)
    A = rng.standard_normal((n, n))
    A[:, 40] = A[:, 3]  # rank deficient
    A[:, 40] -= A[:, 3]
    At = dev(np.ascontiguousarray(A.T))
    with pytest.raises(nb.NebemError) as e:
        nb.solve(At, dev(np.ones(n)))
    assert e.value.code == nb.NEBEM_ESINGULAR


# ------------------------------------------------------- edges and errors

def test_invalid_panel_rejected(nb):
    b = GeometryBuilder()
    b.rect((0, 0, 0), (1e-5, 0, 0), (0, 1e-5, 0))
    g = b.build("bad", Images(), (-1,) * 3, (1,) * 3)
    g.w[0] = [1e-6, 1e-5, 0]  # not perpendicular to u
    with pytest.raises(nb.NebemError) as e:
        gpu_eval(nb, g, np.ones(1), np.zeros((3, 3)))
    assert e.value.code == nb.NEBEM_EINVAL


def test_empty_and_ragged(nb):
    g = parallel_plates(n=3)
    rng = np.random.default_rng(4)
    sigma = rng.normal(size=g.n)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    out = nb.eval_points(dp, dev(sigma), e, e, e)
    assert all(t.numel() == 0 for t in out)
    for m in (1, 255, 257, 1000):
        pts = uniform_points(g.box_lo, g.box_hi, m, m)
        got = gpu_eval(nb, g, sigma, pts)
        ref = oracle.eval_points(g, sigma, pts)
        ephi, eE = rel_errors(got, ref)
        assert ephi < 1e-10 and eE < 1e-10


def test_deterministic_and_batch_independent(nb):
    g = gem_cell().subset(np.arange(0, 8064, 7)).with_images(Images())
    rng = np.random.default_rng(5)
    sigma = rng.normal(size=g.n)
    pts = uniform_points((0, 0, 1e-4), (1.4e-4, 1.2e-4, 1e-3), 3000, 6)
    a = gpu_eval(nb, g, sigma, pts)
    b = gpu_eval(nb, g, sigma, pts)
    assert np.array_equal(a, b)
    c = gpu_eval(nb, g, sigma, pts[1234:1500])
    assert np.array_equal(c, a[1234:1500])


@pytest.mark.parametrize("precision", [0, 1])
def test_morton_ordered_eval_bitwise(nb, precision):
    """Batches of >= 4096 points are evaluated in Morton order of the points
    and scattered back; each point's arithmetic is independent of its wave
    neighbours, so the results equal, bit for bit, those of the same points
    in batches below the threshold (evaluated in the caller's order)."""
    g = gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2)
    rng = np.random.default_rng(21)
    sigma = rng.normal(0, 1e-5, g.n)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    sg = dev(sigma)
    for m in (4096, 4097, 9000):
        pts = uniform_points(g.box_lo, g.box_hi, m, 100 + m)
        pts[17] = pts[3]  # a duplicated point
        big = stack(nb.eval_points(dp, sg, *cols(pts), precision=precision))
        small = np.vstack([stack(nb.eval_points(dp, sg, *cols(pts[k:k + 2000]), precision=precision))
                           for k in range(0, m, 2000)])
        assert np.array_equal(big, small), m
    # all points identical: a box of zero extent
    pts = np.repeat(uniform_points(g.box_lo, g.box_hi, 1, 5), 5000, axis=0)
    big = stack(nb.eval_points(dp, sg, *cols(pts), precision=precision))
    one = stack(nb.eval_points(dp, sg, *cols(pts[:1]), precision=precision))
    assert np.array_equal(big, np.repeat(one, 5000, axis=0))
    # against the oracle on a sample of the ordered batch (FP64 bar / mixed bar)
    pts = uniform_points(g.box_lo, g.box_hi, 6000, 8)
    got = stack(nb.eval_points(dp, sg, *cols(pts), precision=precision))
    idx = rng.choice(len(pts), 24, replace=False)
    ref = oracle.eval_points(g, sigma, pts[idx])
    ephi, eE = rel_errors(got[idx], ref)
    tol = 1e-10 if precision == 0 else 1e-6
    assert ephi < tol and eE < tol, (ephi, eE)


def test_morton_ordered_session(nb):
    """Session evaluation through the ordered path."""
    g = gem_cell(k=16, nr=2, nz_kapton=1, nz_cu=1, nd=2, n_images=2)
    dp = nb.DevicePanels.from_geometry(g, DEV)
    ses = nb.Session(dp, precision=0)
    pts = uniform_points(g.box_lo, g.box_hi, 5000, 3)
    full = stack(ses.eval_points(*cols(pts)))
    parts = np.vstack([stack(ses.eval_points(*cols(pts[k:k + 1000]))) for k in range(0, 5000, 1000)])
    assert np.array_equal(full, parts)
    ref = stack(nb.eval_points(dp, ses.sigma(), *cols(pts), precision=0))
    assert np.array_equal(full, ref)
    ses.close()
