"""FP64 CPU oracle for the neBEM hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (HIP kernels + C-ABI) never calls
it, links it or falls back to it, and it shares no code with that library.

The C part (nebem_oracle.c) holds the panel integrals, evaluation, assembly
and point-charge sums; this module wraps it with ctypes and adds the pieces
that are plain library steps: the dense solve (LAPACK LU with partial
pivoting through scipy, paper Eq. Matrix and Algorithm 1's factorisation)
and the explicit-Euler space-charge step (paper Algorithm 4 with the fixed
drift model described at `spacecharge_step`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nebem_oracle.c")
_LIB = os.path.join(_HERE, "libnebem_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA
    contraction, OpenMP over the independent outer loops)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Images(ctypes.Structure):
    _fields_ = [("a1", ctypes.c_double * 3), ("a2", ctypes.c_double * 3),
                ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("mirror_mask", ctypes.c_int32),
                ("mirror_pos", ctypes.c_double * 3),
                ("mirror_parity", ctypes.c_int32 * 3)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_panel.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P]
    lib.oracle_panel_exact.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P]
    lib.oracle_panel_gauss.argtypes = [ctypes.c_int, P, P, P, P, P]
    lib.oracle_eval.argtypes = [i64, P, P, P, P, P, ctypes.POINTER(_Images), i64, P, P, ctypes.c_int]
    lib.oracle_assemble.argtypes = [i64, P, P, P, P, P, P, P, ctypes.POINTER(_Images), P, P, ctypes.c_int]
    lib.oracle_assemble_rows.argtypes = [i64, P, P, P, P, P, P, P, ctypes.POINTER(_Images), P, i64, P, P,
                                         ctypes.c_int]
    lib.oracle_coulomb.argtypes = [i64, P, P, i64, P, P, P, P, ctypes.c_int]
    lib.oracle_ke.restype = ctypes.c_double
    lib.oracle_eps0.restype = ctypes.c_double
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def ke() -> float:
    return _load().oracle_ke()


def eps0() -> float:
    return _load().oracle_eps0()


def max_threads() -> int:
    return _load().oracle_max_threads()


def _images(img) -> _Images:
    s = _Images()
    if img is None:
        return s
    for k in range(3):
        s.a1[k] = float(img.a1[k])
        s.a2[k] = float(img.a2[k])
        s.mirror_pos[k] = float(img.mirror_pos[k])
        s.mirror_parity[k] = int(img.mirror_parity[k])
    s.n1, s.n2, s.mirror_mask = int(img.n1), int(img.n2), int(img.mirror_mask)
    return s


def panel(kind, o, u, w, p, on_plane=False, method="auto") -> np.ndarray:
    """(Phi', E'x, E'y, E'z) of one unit-density panel at point p."""
    lib = _load()
    out = np.zeros(4)
    o, u, w, p = (_f64(x, 3) for x in (o, u, w, p))
    if method == "auto":
        lib.oracle_panel(int(kind), _p(o), _p(u), _p(w), _p(p), int(on_plane), _p(out))
    elif method == "exact":
        lib.oracle_panel_exact(int(kind), _p(o), _p(u), _p(w), _p(p), int(on_plane), _p(out))
    elif method == "gauss":
        lib.oracle_panel_gauss(int(kind), _p(o), _p(u), _p(w), _p(p), _p(out))
    else:
        raise ValueError(method)
    return out


def eval_points(geom, sigma, pts, nthreads: int = 0) -> np.ndarray:
    """(phi, Ex, Ey, Ez) [m, 4] at points from all panels and their copies."""
    lib = _load()
    pts = _f64(pts, (-1, 3))
    out = np.zeros((pts.shape[0], 4))
    kind = np.ascontiguousarray(geom.kind, dtype=np.int32)
    o, u, w = _f64(geom.o), _f64(geom.u), _f64(geom.w)
    sig = _f64(sigma)
    im = _images(geom.images)
    lib.oracle_eval(geom.n, _p(kind), _p(o), _p(u), _p(w), _p(sig), ctypes.byref(im),
                    pts.shape[0], _p(pts), _p(out), int(nthreads))
    return out


def assemble(geom, colloc=None, nthreads: int = 0) -> np.ndarray:
    """Influence matrix, column-major storage returned as a Fortran-ordered
    [n, n] array A with A[i, j] = influence of panel j at collocation i."""
    lib = _load()
    n = geom.n
    A = np.zeros(n * n)
    kind = np.ascontiguousarray(geom.kind, dtype=np.int32)
    bc = np.ascontiguousarray(geom.bc, dtype=np.int32)
    o, u, w = _f64(geom.o), _f64(geom.u), _f64(geom.w)
    ep, en = _f64(geom.eps_pos), _f64(geom.eps_neg)
    c = None if colloc is None else _f64(colloc, (-1, 3))
    im = _images(geom.images)
    lib.oracle_assemble(n, _p(kind), _p(o), _p(u), _p(w), _p(bc), _p(ep), _p(en), ctypes.byref(im),
                        _p(c), _p(A), int(nthreads))
    return A.reshape((n, n), order="F")


def assemble_rows(geom, rows, colloc=None, nthreads: int = 0) -> np.ndarray:
    """Selected rows of the influence matrix, [len(rows), n]."""
    lib = _load()
    n = geom.n
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((rows.shape[0], n))
    kind = np.ascontiguousarray(geom.kind, dtype=np.int32)
    bc = np.ascontiguousarray(geom.bc, dtype=np.int32)
    o, u, w = _f64(geom.o), _f64(geom.u), _f64(geom.w)
    ep, en = _f64(geom.eps_pos), _f64(geom.eps_neg)
    c = None if colloc is None else _f64(colloc, (-1, 3))
    im = _images(geom.images)
    lib.oracle_assemble_rows(n, _p(kind), _p(o), _p(u), _p(w), _p(bc), _p(ep), _p(en), ctypes.byref(im),
                             _p(c), rows.shape[0], _p(rows), _p(out), int(nthreads))
    return out


def coulomb(targets, sources, q, self_index=None, nthreads: int = 0, with_abs: bool = False):
    """(phi, E) [nt, 4] of point charges at targets, skipping self pairs and
    coincident charges; with_abs: also the sum of the field terms'
    magnitudes, k_e sum_j |q_j| / r_j^2 [nt] (the scale of a
    condition-normalised error)."""
    lib = _load()
    t = _f64(targets, (-1, 3))
    s = _f64(sources, (-1, 3))
    qq = _f64(q)
    si = None if self_index is None else np.ascontiguousarray(self_index, dtype=np.int64)
    out = np.zeros((t.shape[0], 4))
    ab = np.zeros(t.shape[0]) if with_abs else None
    lib.oracle_coulomb(t.shape[0], _p(t), _p(si), s.shape[0], _p(s), _p(qq), _p(out), _p(ab), int(nthreads))
    return (out, ab) if with_abs else out


def solve(A, b):
    """sigma solving A sigma = b by LU with partial pivoting (LAPACK getrf /
    getrs via scipy).  The paper forms K^-1 (Algorithm 1) and multiplies;
    the solution is the same vector."""
    import scipy.linalg as sla
    lu, piv = sla.lu_factor(A)
    return sla.lu_solve((lu, piv), b)


def solve_refined(A, b, steps: int = 2):
    """`solve` followed by `steps` rounds of iterative refinement in FP64
    (r = b - A sigma, sigma += A^-1 r with the same LU factors): the same
    definition, sigma solving A sigma = b, with the LU solution's residual
    (which an ill-conditioned collocation matrix makes large: 7e-11 relative
    on the 8064-element GEM cell) brought down to the rounding of the
    residual product itself."""
    import scipy.linalg as sla
    lu, piv = sla.lu_factor(A)
    x = sla.lu_solve((lu, piv), b)
    for _ in range(steps):
        x = x + sla.lu_solve((lu, piv), b - A @ x)
    return x


def primitive_density(elems, prims, elem_prim, sigma) -> np.ndarray:
    """Adaptive Modelling's simplified representation (Sec. 3): each
    primitive's average density, its elements' total charge over its own
    area, sum_{j in p} sigma_j A_j / A_p."""
    def areas(g):
        a = np.linalg.norm(np.cross(g.u, g.w), axis=1)
        return np.where(np.asarray(g.kind) == 1, 0.5 * a, a)
    q = np.zeros(prims.n)
    np.add.at(q, np.asarray(elem_prim), np.asarray(sigma) * areas(elems))
    return q / areas(prims)


def eval_adaptive(elems, prims, elem_prim, prim_after, sigma, pts, nthreads: int = 0) -> np.ndarray:
    """Adaptive Modelling as defined: translated copies with |i1|, |i2| <=
    prim_after (every reflection) element by element, every farther copy
    primitive by primitive with `primitive_density`; prim_after < 0: no
    simplification.  Written as three plain evaluations: elements over the
    inner lattice, plus primitives over the full lattice, minus primitives
    over the inner lattice."""
    im = elems.images
    if prim_after < 0 or (prim_after >= im.n1 and prim_after >= im.n2):
        return eval_points(elems.with_images(_inner(im, prim_after if prim_after >= 0 else max(im.n1, im.n2))),
                           sigma, pts, nthreads)
    inner = _inner(im, prim_after)
    sbar = primitive_density(elems, prims, elem_prim, sigma)
    return (eval_points(elems.with_images(inner), sigma, pts, nthreads)
            + eval_points(prims.with_images(im), sbar, pts, nthreads)
            - eval_points(prims.with_images(inner), sbar, pts, nthreads))


def _inner(im, k):
    import dataclasses
    return dataclasses.replace(im, n1=min(im.n1, k), n2=min(im.n2, k))


def voxel_lines(xyz, q, origin, step, shape, placement: str = "centre"):
    """Point charges reduced to line charges (Algorithm 3): charges binned
    into the voxels of a regular grid (voxel (i, j, k) = floor((x - origin)
    / step) per axis, index i + nx (j + ny k); charges outside dropped);
    every occupied voxel becomes one segment parallel to z over the voxel's
    z extent, carrying the voxel's total charge uniformly.  The voxel record
    of Algorithm 3 holds only the total charge and the occupancy, so by
    default (placement "centre") the segment runs through the voxel's
    centre in x, y; placement "weighted" puts it at the |q|-weighted mean
    x, y of the voxel's charges instead.  Returns (lines (L, 7): ax, ay,
    az, bx, by, bz, lambda, in increasing voxel index; number of charges
    outside)."""
    if placement not in ("centre", "weighted"):
        raise ValueError(placement)
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    origin, step = np.asarray(origin, dtype=np.float64), np.asarray(step, dtype=np.float64)
    shape = np.asarray(shape)
    ijk = np.floor((xyz - origin) / step).astype(np.int64)
    inside = np.all((ijk >= 0) & (ijk < shape), axis=1)
    ijk, xyz, q = ijk[inside], xyz[inside], q[inside]
    key = ijk[:, 0] + shape[0] * (ijk[:, 1] + shape[1] * ijk[:, 2])
    vox, inv = np.unique(key, return_inverse=True)
    Q = np.bincount(inv, q, len(vox))
    i = vox % shape[0]
    j = (vox // shape[0]) % shape[1]
    k = vox // (shape[0] * shape[1])
    x = origin[0] + (i + 0.5) * step[0]
    y = origin[1] + (j + 0.5) * step[1]
    if placement == "weighted":
        W = np.bincount(inv, np.abs(q), len(vox))
        cx = np.bincount(inv, np.abs(q) * xyz[:, 0], len(vox))
        cy = np.bincount(inv, np.abs(q) * xyz[:, 1], len(vox))
        x = np.where(W > 0, cx / np.where(W > 0, W, 1), x)
        y = np.where(W > 0, cy / np.where(W > 0, W, 1), y)
    z0 = origin[2] + k * step[2]
    lines = np.column_stack([x, y, z0, x, y, z0 + step[2], Q / step[2]])
    return lines, int((~inside).sum())


def line_field(lines, pts) -> np.ndarray:
    """(phi, Ex, Ey, Ez) at the points of uniformly charged segments (A, B,
    lambda): with t the unit direction, s_a = (a - P).t, rho the distance of
    P from the line,
      phi = k_e lambda (asinh(s_B / rho) - asinh(s_A / rho)),
      E   = k_e lambda [ (s_B/r_B - s_A/r_A) (P - F) / rho^2 + (1/r_B - 1/r_A) t ],
    F the foot of P on the line (the integral of (P - X)/|P - X|^3 along the
    segment).  Plain loops over the segments."""
    lines = np.asarray(lines, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros((len(pts), 4))
    for a0, a1, a2, b0, b1, b2, lam in lines:
        A, B = np.array([a0, a1, a2]), np.array([b0, b1, b2])
        L = np.linalg.norm(B - A)
        t = (B - A) / L
        d = pts - A
        along = d @ t
        perp = d - along[:, None] * t
        rho2 = (perp * perp).sum(axis=1)
        rho = np.sqrt(rho2)
        sA, sB = -along, L - along
        rA, rB = np.linalg.norm(pts - A, axis=1), np.linalg.norm(pts - B, axis=1)
        out[:, 0] += ke() * lam * (np.arcsinh(sB / rho) - np.arcsinh(sA / rho))
        g = (sB / rB - sA / rA) / rho2
        out[:, 1:] += ke() * lam * (g[:, None] * perp + (1.0 / rB - 1.0 / rA)[:, None] * t)
    return out


def charge_field_lines(xyz, q, origin, step, shape, placement: str = "centre"):
    """The charges' own field at every charge with the charges reduced to
    line charges (Algorithm 3 as the space-charge source, Sec. 4.2), near
    voxels excepted: a charge in voxel (i, j, k) feels the lines (from
    `voxel_lines`) of all voxels outside i +- 1, j +- 1, k +- 1, and the
    charges of those 27 voxels one by one (k_e q_j (x - x_j)/|x - x_j|^3,
    coincident charges skipped); a charge outside the grid feels every line.
    Returns (E (n, 3), S (n,)) with S the sum of the magnitudes of all terms
    (the scale of a condition-normalised error).  Plain loops over lines."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    lines, _ = voxel_lines(xyz, q, origin, step, shape, placement)
    origin, step = np.asarray(origin, dtype=np.float64), np.asarray(step, dtype=np.float64)
    shape = np.asarray(shape)
    ijk = np.floor((xyz - origin) / step).astype(np.int64)
    inside = np.all((ijk >= 0) & (ijk < shape), axis=1)
    key = np.where(inside, ijk[:, 0] + shape[0] * (ijk[:, 1] + shape[1] * ijk[:, 2]), -1)
    vox = np.unique(key[inside])  # the lines' voxels, in line order
    vijk = np.column_stack([vox % shape[0], (vox // shape[0]) % shape[1], vox // (shape[0] * shape[1])])
    n = len(xyz)
    E = np.zeros((n, 3))
    S = np.zeros(n)
    for l in range(len(lines)):
        near = inside & np.all(np.abs(ijk - vijk[l]) <= 1, axis=1)
        far = ~near
        if far.any():
            with np.errstate(divide="ignore", invalid="ignore"):
                f = line_field(lines[l:l + 1], xyz[far])[:, 1:]
            E[far] += f
            S[far] += np.linalg.norm(f, axis=1)
    for i in np.flatnonzero(inside):
        nb = inside & np.all(np.abs(ijk - ijk[i]) <= 1, axis=1)
        d = xyz[i] - xyz[nb]
        r2 = (d * d).sum(axis=1)
        ok = r2 > 0
        t = ke() * q[nb][ok, None] * d[ok] / (r2[ok] * np.sqrt(r2[ok]))[:, None]
        E[i] += t.sum(axis=0)
        S[i] += np.linalg.norm(t, axis=1).sum()
    return E, S


def grid_nodes(origin, step, shape) -> np.ndarray:
    """Coordinates (nx*ny*nz, 3) of a regular grid's nodes, node (i, j, k)
    at row i + nx (j + ny k): the FastVolume grid of Sec. 3 (a volume
    sampled once, then interpolated)."""
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.column_stack([origin[0] + i.ravel() * step[0], origin[1] + j.ravel() * step[1],
                            origin[2] + k.ravel() * step[2]])


def trilinear(origin, step, shape, values, pts) -> np.ndarray:
    """Trilinear interpolation of node values (nx*ny*nz, c), node order as in
    `grid_nodes`, at points (m, 3): on each axis the cell index is
    floor((x - origin)/step), limited to [0, n-2], and the weights are the
    fractional distances to the cell's two faces.  Points outside the grid
    (any coordinate below the first or above the last node) give NaN.
    Plain loops over the 8 corners; the definition, not a fast path."""
    pts = np.asarray(pts, dtype=np.float64)
    values = np.asarray(values, dtype=np.float64)
    nx, ny, nz = shape
    u = (pts - np.asarray(origin)) / np.asarray(step)
    n = np.array([nx, ny, nz])
    inside = np.all((u >= 0) & (u <= n - 1), axis=1)
    i0 = np.clip(np.floor(u).astype(np.int64), 0, n - 2)
    f = u - i0
    out = np.zeros((len(pts), values.shape[1]))
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                w = ((f[:, 0] if di else 1 - f[:, 0]) * (f[:, 1] if dj else 1 - f[:, 1])
                     * (f[:, 2] if dk else 1 - f[:, 2]))
                idx = (i0[:, 0] + di) + nx * ((i0[:, 1] + dj) + ny * (i0[:, 2] + dk))
                out += w[:, None] * values[np.where(inside, idx, 0)]
    out[~inside] = np.nan
    return out


def axes_nodes(axes) -> np.ndarray:
    """Nodes (nx*ny*nz, 3) of a graded grid given by three strictly
    increasing coordinate lists, node (i, j, k) at row i + nx (j + ny k)."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in axes)
    k, j, i = np.meshgrid(np.arange(len(z)), np.arange(len(y)), np.arange(len(x)), indexing="ij")
    return np.column_stack([x[i.ravel()], y[j.ravel()], z[k.ravel()]])


def trilinear_axes(axes, values, pts) -> np.ndarray:
    """Trilinear interpolation on a graded grid (FastVolume with nodes dense
    where the field varies fast): on each axis the cell is the last node at
    or below the coordinate (the last cell for the last node), the weight
    the fractional position (x - a_i) / (a_{i+1} - a_i); outside
    [first node, last node] on any axis: NaN.  Plain loops over the 8
    corners."""
    ax = [np.asarray(a, dtype=np.float64) for a in axes]
    pts = np.asarray(pts, dtype=np.float64)
    values = np.asarray(values, dtype=np.float64)
    n = [len(a) for a in ax]
    i0, f = [], []
    inside = np.ones(len(pts), dtype=bool)
    for d in range(3):
        a, x = ax[d], pts[:, d]
        inside &= (x >= a[0]) & (x <= a[-1])
        i = np.clip(np.searchsorted(a, x, side="right") - 1, 0, n[d] - 2)
        i0.append(i)
        f.append((x - a[i]) / (a[i + 1] - a[i]))
    out = np.zeros((len(pts), values.shape[1]))
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                w = ((f[0] if di else 1 - f[0]) * (f[1] if dj else 1 - f[1]) * (f[2] if dk else 1 - f[2]))
                idx = (i0[0] + di) + n[0] * ((i0[1] + dj) + n[1] * (i0[2] + dk))
                out += w[:, None] * values[np.where(inside, idx, 0)]
    out[~inside] = np.nan
    return out


def rhs_with_charges(geom, b0, qxyz, q, nthreads: int = 0) -> np.ndarray:
    """Boundary values with the known charges moved to the right-hand side
    (paper Sec. 4.1, RHVector with the known-charge contribution):
    conductor rows V_i - phi_q(c_i), dielectric rows -n_i . E_q(c_i)."""
    c = geom.centroids()
    f = coulomb(c, qxyz, q, None, nthreads)
    n = geom.normals()
    en = np.einsum("ij,ij->i", f[:, 1:], n)
    return np.where(geom.bc == 0, b0 - f[:, 0], -en)


@dataclass
class SpaceChargeParams:
    dt: float = 1e-12          # s
    mobility: float = 1e-4     # m^2 / (V s), same for both signs
    resolve_every: int = 10
    threshold: float = -1.0    # >= 0: Algorithm 4's SpChTh on sum |q| instead of the schedule


def spacecharge_step(geom, A, b0, sigma, qxyz, q, step_index, params: SpaceChargeParams,
                     nthreads: int = 0):
    """One step of the dynamic space-charge loop (paper Algorithm 4 with a
    fixed drift model in place of the avalanche transport):
      1. if a re-solve is due -- step_index % resolve_every == 0, or with
         threshold >= 0 (Algorithm 4's SpChTh) when the charges' magnitude
         sum |q| exceeds the threshold -- re-solve sigma with the charges on
         the right-hand side (LU with FP64 refinement: the unrefined
         solution's residual moves the field by ~1e-6 relative at the
         weak-field points of a GEM cell);
      2. E at every charge = panel part (all copies) + point-charge part
         (all other charges, no copies);
      3. every charge moves by sign(q) * mobility * E * dt (all fields from
         the start-of-step positions).
    Returns (new positions, sigma, E at the charges)."""
    if params.threshold >= 0.0:
        due = float(np.abs(q).sum()) > params.threshold
    else:
        due = step_index % params.resolve_every == 0
    if due:
        b = rhs_with_charges(geom, b0, qxyz, q, nthreads)
        sigma = solve_refined(A, b)
    ep = eval_points(geom, sigma, qxyz, nthreads)[:, 1:]
    ec = coulomb(qxyz, qxyz, q, np.arange(qxyz.shape[0]), nthreads)[:, 1:]
    E = ep + ec
    new = qxyz + (np.sign(q) * params.mobility * params.dt)[:, None] * E
    return new, sigma, E
