"""Python binding of libnebem (the C-ABI declared in include/nebem.h).

Argument marshalling only: torch tensors provide device memory and streams,
every step of the computation runs in the library's HIP kernels.  The
library must be built (``__graft_entry__.build()``); importing this package
without it raises ImportError -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnebem.so")

NEBEM_OK = 0
NEBEM_EINVAL = -1
NEBEM_ENOMEM = -2
NEBEM_ESINGULAR = -3
NEBEM_ENOCONV = -4
NEBEM_EDEVICE = -5
NEBEM_EBUSY = -6
FP64 = 0
MIXED = 1

EXPORTED = (
    "nebem_default_options", "nebem_assemble", "nebem_solve", "nebem_solve_factored", "nebem_norm1",
    "nebem_condest", "nebem_eval", "nebem_eval_multi", "nebem_eval_adaptive", "nebem_fastvol_build",
    "nebem_fastvol_interp", "nebem_fastvol_build_axes", "nebem_fastvol_interp_axes",
    "nebem_voxelize_charges", "nebem_line_field",
    "nebem_session_create", "nebem_session_destroy", "nebem_session_n", "nebem_session_sigma",
    "nebem_session_solve", "nebem_session_condest", "nebem_session_eval", "nebem_session_eval_noalloc", "nebem_session_fastvol",
    "nebem_spacecharge_step",
    "nebem_spacecharge_step_lines", "nebem_charge_field_lines",
    "nebem_last_error",
    "nebem_server_default_options", "nebem_server_create", "nebem_server_submit", "nebem_server_wait",
    "nebem_server_stats", "nebem_server_destroy",
)


class NebemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nebem error {code}: {msg}")
        self.code = code


class Panels(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("kind", ctypes.c_void_p),
                ("ox", ctypes.c_void_p), ("oy", ctypes.c_void_p), ("oz", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("uz", ctypes.c_void_p),
                ("wx", ctypes.c_void_p), ("wy", ctypes.c_void_p), ("wz", ctypes.c_void_p),
                ("bc", ctypes.c_void_p), ("value", ctypes.c_void_p),
                ("eps_pos", ctypes.c_void_p), ("eps_neg", ctypes.c_void_p)]


class ImagesC(ctypes.Structure):
    _fields_ = [("a1", ctypes.c_double * 3), ("a2", ctypes.c_double * 3),
                ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("mirror_mask", ctypes.c_int32),
                ("mirror_pos", ctypes.c_double * 3), ("mirror_parity", ctypes.c_int32 * 3)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("near_factor", ctypes.c_double),
                ("ir_tol", ctypes.c_double), ("ir_max_iter", ctypes.c_int32),
                ("sc_dt", ctypes.c_double), ("sc_mobility", ctypes.c_double),
                ("sc_resolve_every", ctypes.c_int32), ("sc_threshold", ctypes.c_double)]


class GridC(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("step", ctypes.c_double * 3), ("n", ctypes.c_int32 * 3)]


class AxesC(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("n", ctypes.c_int32 * 3)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int32), ("rel_resid", ctypes.c_double)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("batch_interactions", ctypes.c_double),
                ("max_items", ctypes.c_int32), ("large_interactions", ctypes.c_double),
                ("max_large", ctypes.c_int32)]


class RequestStats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("points", ctypes.c_int64)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("points_done", ctypes.c_int64),
                ("interactions", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("queued", ctypes.c_int64), ("active", ctypes.c_int64),
                ("backfilled", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    PP, PI, PO = ctypes.POINTER(Panels), ctypes.POINTER(ImagesC), ctypes.POINTER(Options)
    lib.nebem_default_options.argtypes = [PO]
    lib.nebem_default_options.restype = None
    lib.nebem_last_error.restype = ctypes.c_char_p
    lib.nebem_assemble.argtypes = [PP, PI, P, P, P, PO, P, P]
    lib.nebem_solve.argtypes = [P, i64, P, i64, P, P, PO, ctypes.POINTER(SolveInfo), P]
    lib.nebem_solve_factored.argtypes = [P, P, i64, P, i64, P, P]
    lib.nebem_eval.argtypes = [PP, PI, P, P, P, P, i64, P, P, P, P, PO, P]
    lib.nebem_eval_adaptive.argtypes = [PP, PP, P, i32, PI, P, P, P, P, i64, P, P, P, P, PO, P]
    lib.nebem_eval_adaptive.restype = i32
    PG = ctypes.POINTER(GridC)
    PA = ctypes.POINTER(AxesC)
    lib.nebem_fastvol_build_axes.argtypes = [PP, PI, P, PA, P, PO, P]
    lib.nebem_fastvol_build_axes.restype = i32
    lib.nebem_fastvol_interp_axes.argtypes = [PA, P, P, P, P, i64, P, P, P, P, P]
    lib.nebem_fastvol_interp_axes.restype = i32
    lib.nebem_voxelize_charges.argtypes = [P, P, P, P, i64, PG, i32, P, i64, ctypes.POINTER(i64),
                                           ctypes.POINTER(i64), P]
    lib.nebem_voxelize_charges.restype = i32
    lib.nebem_line_field.argtypes = [P, i64, P, P, P, i64, P, P, P, P, P]
    lib.nebem_line_field.restype = i32
    lib.nebem_fastvol_build.argtypes = [PP, PI, P, PG, P, PO, P]
    lib.nebem_fastvol_build.restype = i32
    lib.nebem_fastvol_interp.argtypes = [PG, P, P, P, P, i64, P, P, P, P, P]
    lib.nebem_fastvol_interp.restype = i32
    lib.nebem_eval_multi.argtypes = [PP, PI, P, i64, P, P, P, i64, P, P, P, P, PO, P]
    lib.nebem_eval_multi.restype = i32
    lib.nebem_norm1.argtypes = [P, i64, ctypes.POINTER(ctypes.c_double), P]
    lib.nebem_norm1.restype = i32
    lib.nebem_condest.argtypes = [P, P, i64, ctypes.c_double, ctypes.POINTER(ctypes.c_double), P]
    lib.nebem_condest.restype = i32
    lib.nebem_session_condest.argtypes = [P, ctypes.POINTER(ctypes.c_double), P]
    lib.nebem_session_condest.restype = i32
    for name in ("nebem_assemble", "nebem_solve", "nebem_solve_factored", "nebem_eval"):
        getattr(lib, name).restype = i32
    lib.nebem_session_create.argtypes = [PP, PI, PO, P, ctypes.POINTER(P)]
    lib.nebem_session_create.restype = i32
    lib.nebem_session_destroy.argtypes = [P]
    lib.nebem_session_destroy.restype = None
    lib.nebem_session_n.argtypes = [P]
    lib.nebem_session_n.restype = i64
    lib.nebem_session_sigma.argtypes = [P]
    lib.nebem_session_sigma.restype = P
    lib.nebem_session_solve.argtypes = [P, P, ctypes.POINTER(SolveInfo), P]
    lib.nebem_session_solve.restype = i32
    lib.nebem_session_eval.argtypes = [P, P, P, P, i64, P, P, P, P, P]
    lib.nebem_session_eval.restype = i32
    lib.nebem_session_fastvol.argtypes = [P, PG, PA, P, P]
    lib.nebem_session_fastvol.restype = i32
    lib.nebem_session_eval_noalloc.argtypes = [P, P, P, P, i64, P, P, P, P, P]
    lib.nebem_session_eval_noalloc.restype = i32
    lib.nebem_spacecharge_step.argtypes = [P, P, P, P, P, i64, i32, P, P, P, P]
    lib.nebem_spacecharge_step.restype = i32
    lib.nebem_charge_field_lines.argtypes = [P, P, P, P, i64, PG, i32, P, P, P, ctypes.POINTER(i64), P]
    lib.nebem_charge_field_lines.restype = i32
    lib.nebem_spacecharge_step_lines.argtypes = [P, P, P, P, P, i64, i32, ctypes.POINTER(GridC), i32, P, P, P,
                                                 ctypes.POINTER(i64), P]
    lib.nebem_spacecharge_step_lines.restype = i32
    lib.nebem_server_default_options.argtypes = [ctypes.POINTER(ServerOptions)]
    lib.nebem_server_default_options.restype = None
    lib.nebem_server_create.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]
    lib.nebem_server_create.restype = i32
    lib.nebem_server_submit.argtypes = [P, i32, P, P, P, i64, P, P, P, P, ctypes.POINTER(i64)]
    lib.nebem_server_submit.restype = i32
    lib.nebem_server_wait.argtypes = [P, i64, ctypes.POINTER(RequestStats)]
    lib.nebem_server_wait.restype = i32
    lib.nebem_server_stats.argtypes = [P, ctypes.POINTER(ServerCounters)]
    lib.nebem_server_stats.restype = i32
    lib.nebem_server_destroy.argtypes = [P]
    lib.nebem_server_destroy.restype = None
    return lib


lib = _load()


def _check(code):
    if code != NEBEM_OK:
        raise NebemError(code, lib.nebem_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def options(precision=FP64, **kw) -> Options:
    o = Options()
    lib.nebem_default_options(ctypes.byref(o))
    o.precision = precision
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def images_struct(img) -> ImagesC:
    s = ImagesC()
    if img is None:
        return s
    for k in range(3):
        s.a1[k] = float(img.a1[k])
        s.a2[k] = float(img.a2[k])
        s.mirror_pos[k] = float(img.mirror_pos[k])
        s.mirror_parity[k] = int(img.mirror_parity[k])
    s.n1, s.n2, s.mirror_mask = int(img.n1), int(img.n2), int(img.mirror_mask)
    return s


@dataclass
class DevicePanels:
    """A geometry's panel arrays resident on the GPU, plus the C struct that
    points at them."""
    tensors: dict
    n: int
    images: object
    struct: Panels

    @classmethod
    def from_geometry(cls, geom, device="cuda"):
        import torch
        soa = geom.soa()
        t = {}
        for k, v in soa.items():
            dt = torch.int32 if v.dtype == np.int32 else torch.float64
            t[k] = torch.from_numpy(np.ascontiguousarray(v)).to(device=device, dtype=dt)
        s = Panels()
        s.n = geom.n
        for k in ("kind", "ox", "oy", "oz", "ux", "uy", "uz", "wx", "wy", "wz", "bc", "value",
                  "eps_pos", "eps_neg"):
            setattr(s, k, t[k].data_ptr())
        return cls(t, geom.n, geom.images, s)


def assemble(dp: DevicePanels, A=None, colloc=None, precision=FP64, stream=None, **opt):
    """Influence matrix (n x n, column-major in a torch float64 tensor of
    shape (n, n) whose storage is the transpose: A_t[j, i] = A[i, j])."""
    import torch
    n = dp.n
    if A is None:
        A = torch.empty((n, n), dtype=torch.float64, device=dp.tensors["ox"].device)
    im = images_struct(dp.images)
    o = options(precision, **opt)
    cx = cy = cz = None
    if colloc is not None:
        cx, cy, cz = colloc
    _check(lib.nebem_assemble(ctypes.byref(dp.struct), ctypes.byref(im), _ptr(cx), _ptr(cy), _ptr(cz),
                              ctypes.byref(o), _ptr(A), _stream(stream)))
    return A


def solve(A, b, precision=FP64, stream=None, sigma=None, ipiv=None, **opt):
    """sigma = A^-1 b.  A: (n, n) float64 tensor holding the column-major
    matrix (as returned by `assemble`); FP64 mode overwrites it with the LU
    factors.  b: (n,) or (nrhs, n) float64.  Returns (sigma, ipiv, info)."""
    import torch
    n = A.shape[0]
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    if sigma is None:
        sigma = torch.empty_like(b)
    if ipiv is None:
        ipiv = torch.empty(n, dtype=torch.int32, device=A.device)
    info = SolveInfo()
    o = options(precision, **opt)
    _check(lib.nebem_solve(_ptr(A), n, _ptr(b), nrhs, _ptr(sigma), _ptr(ipiv), ctypes.byref(o),
                           ctypes.byref(info), _stream(stream)))
    return sigma, ipiv, info


def solve_factored(LU, ipiv, b, stream=None, sigma=None):
    import torch
    n = LU.shape[0]
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    if sigma is None:
        sigma = torch.empty_like(b)
    _check(lib.nebem_solve_factored(_ptr(LU), _ptr(ipiv), n, _ptr(b), nrhs, _ptr(sigma), _stream(stream)))
    return sigma


def eval_points_multi(dp: DevicePanels, sigma, px, py, pz, precision=FP64, stream=None, **opt):
    """Weighting fields: sigma is (nsig, n) float64 (row k = density column
    k); returns (phi, ex, ey, ez), each (nsig, m)."""
    import torch
    m = px.shape[0]
    nsig = sigma.shape[0]
    out = [torch.empty((nsig, m), dtype=torch.float64, device=px.device) for _ in range(4)]
    im = images_struct(dp.images)
    o = options(precision, **opt)
    _check(lib.nebem_eval_multi(ctypes.byref(dp.struct), ctypes.byref(im), _ptr(sigma), nsig, _ptr(px), _ptr(py),
                                _ptr(pz), m, *(_ptr(t) for t in out), ctypes.byref(o), _stream(stream)))
    return tuple(out)


def eval_points_adaptive(dp: DevicePanels, dprims: DevicePanels, elem_prim, prim_after, sigma, px, py, pz,
                         precision=FP64, stream=None, **opt):
    """Adaptive Modelling: copies beyond `prim_after` lattice steps summed
    primitive by primitive with primitive-averaged densities.  elem_prim:
    int32 device tensor (n,).  Returns (phi, ex, ey, ez)."""
    import torch
    m = px.shape[0]
    out = [torch.empty(m, dtype=torch.float64, device=px.device) for _ in range(4)]
    im = images_struct(dp.images)
    o = options(precision, **opt)
    _check(lib.nebem_eval_adaptive(ctypes.byref(dp.struct), ctypes.byref(dprims.struct), _ptr(elem_prim),
                                   int(prim_after), ctypes.byref(im), _ptr(sigma), _ptr(px), _ptr(py), _ptr(pz), m,
                                   *(_ptr(t) for t in out), ctypes.byref(o), _stream(stream)))
    return tuple(out)


def grid_struct(origin, step, shape) -> GridC:
    g = GridC()
    for a in range(3):
        g.origin[a], g.step[a], g.n[a] = float(origin[a]), float(step[a]), int(shape[a])
    return g


def fastvol_build(dp: DevicePanels, sigma, origin, step, shape, precision=FP64, stream=None, **opt):
    """phi/E at every node of the grid, interleaved (nx*ny*nz, 4) float64."""
    import torch
    g = grid_struct(origin, step, shape)
    values = torch.empty((int(np.prod(shape)), 4), dtype=torch.float64, device=sigma.device)
    im = images_struct(dp.images)
    o = options(precision, **opt)
    _check(lib.nebem_fastvol_build(ctypes.byref(dp.struct), ctypes.byref(im), _ptr(sigma), ctypes.byref(g),
                                   _ptr(values), ctypes.byref(o), _stream(stream)))
    return values


def fastvol_interp(values, origin, step, shape, px, py, pz, stream=None):
    """Trilinear interpolation of `fastvol_build` values; NaN outside."""
    import torch
    g = grid_struct(origin, step, shape)
    m = px.shape[0]
    out = [torch.empty(m, dtype=torch.float64, device=px.device) for _ in range(4)]
    _check(lib.nebem_fastvol_interp(ctypes.byref(g), _ptr(values), _ptr(px), _ptr(py), _ptr(pz), m,
                                    *(_ptr(t) for t in out), _stream(stream)))
    return tuple(out)


def axes_struct(ax, ay, az) -> AxesC:
    """Graded grid from three strictly increasing float64 device tensors."""
    g = AxesC()
    g.x, g.y, g.z = _ptr(ax), _ptr(ay), _ptr(az)
    g.n[:] = [int(ax.shape[0]), int(ay.shape[0]), int(az.shape[0])]
    return g


def fastvol_build_axes(dp: DevicePanels, sigma, ax, ay, az, precision=FP64, stream=None, **opt):
    """phi/E at every node of a graded grid, interleaved (nx*ny*nz, 4) float64."""
    import torch
    g = axes_struct(ax, ay, az)
    nn = ax.shape[0] * ay.shape[0] * az.shape[0]
    vals = torch.empty((nn, 4), dtype=torch.float64, device=ax.device)
    im = images_struct(dp.images)
    o = options(precision, **opt)
    _check(lib.nebem_fastvol_build_axes(ctypes.byref(dp.struct), ctypes.byref(im), _ptr(sigma), ctypes.byref(g),
                                        _ptr(vals), ctypes.byref(o), _stream(stream)))
    return vals


def fastvol_interp_axes(values, ax, ay, az, px, py, pz, stream=None):
    import torch
    g = axes_struct(ax, ay, az)
    m = px.shape[0]
    out = [torch.empty(m, dtype=torch.float64, device=px.device) for _ in range(4)]
    _check(lib.nebem_fastvol_interp_axes(ctypes.byref(g), _ptr(values), _ptr(px), _ptr(py), _ptr(pz), m,
                                         *(_ptr(t) for t in out), _stream(stream)))
    return tuple(out)


LINE_CENTRE, LINE_WEIGHTED = 0, 1
_PLACEMENT = {"centre": LINE_CENTRE, "weighted": LINE_WEIGHTED}


def voxelize_charges(qx, qy, qz, q, origin, step, shape, placement="centre", stream=None):
    """Line charges (L, 7) from point charges (Algorithm 3) and the number
    of charges outside the voxel grid; placement "centre" (through the voxel
    centre) or "weighted" (at the |q|-weighted mean x, y)."""
    import torch
    g = grid_struct(origin, step, shape)
    pl = _PLACEMENT[placement]
    nl, out = ctypes.c_int64(), ctypes.c_int64()
    code = lib.nebem_voxelize_charges(_ptr(qx), _ptr(qy), _ptr(qz), _ptr(q), qx.shape[0], ctypes.byref(g), pl, None,
                                      0, ctypes.byref(nl), ctypes.byref(out), _stream(stream))
    if code not in (NEBEM_OK, NEBEM_EINVAL) or (code == NEBEM_EINVAL and nl.value == 0):
        _check(code)
    lines = torch.empty((max(nl.value, 1), 7), dtype=torch.float64, device=qx.device)
    _check(lib.nebem_voxelize_charges(_ptr(qx), _ptr(qy), _ptr(qz), _ptr(q), qx.shape[0], ctypes.byref(g), pl,
                                      _ptr(lines), nl.value, ctypes.byref(nl), ctypes.byref(out), _stream(stream)))
    return lines[:nl.value], out.value


def charge_field_lines(qx, qy, qz, q, origin, step, shape, placement="centre", stream=None):
    """The charges' own field at every charge with far voxels as line
    charges and the 27 voxels around each charge as point charges; returns
    ((ex, ey, ez), number of lines)."""
    import torch
    g = grid_struct(origin, step, shape)
    n = qx.shape[0]
    out = [torch.empty(n, dtype=torch.float64, device=qx.device) for _ in range(3)]
    nl = ctypes.c_int64()
    _check(lib.nebem_charge_field_lines(_ptr(qx), _ptr(qy), _ptr(qz), _ptr(q), n, ctypes.byref(g),
                                        _PLACEMENT[placement], *(_ptr(t) for t in out), ctypes.byref(nl),
                                        _stream(stream)))
    return tuple(out), nl.value


def line_field(lines, px, py, pz, stream=None):
    """(phi, ex, ey, ez) of uniformly charged segments at the points."""
    import torch
    m = px.shape[0]
    out = [torch.empty(m, dtype=torch.float64, device=px.device) for _ in range(4)]
    _check(lib.nebem_line_field(_ptr(lines), lines.shape[0], _ptr(px), _ptr(py), _ptr(pz), m,
                                *(_ptr(t) for t in out), _stream(stream)))
    return tuple(out)


def norm1(A, stream=None):
    """||A||_1 of the column-major matrix held by A (as from `assemble`)."""
    out = ctypes.c_double()
    _check(lib.nebem_norm1(_ptr(A), A.shape[0], ctypes.byref(out), _stream(stream)))
    return out.value


def condest(LU, ipiv, anorm, stream=None):
    """cond_1 estimate from FP64 factors (`solve`) and ||A||_1 (`norm1`)."""
    out = ctypes.c_double()
    _check(lib.nebem_condest(_ptr(LU), _ptr(ipiv), LU.shape[0], float(anorm), ctypes.byref(out), _stream(stream)))
    return out.value


def eval_points(dp: DevicePanels, sigma, px, py, pz, precision=FP64, stream=None, out=None, **opt):
    """(phi, ex, ey, ez) float64 tensors at the points."""
    import torch
    m = px.shape[0]
    if out is None:
        out = tuple(torch.empty(m, dtype=torch.float64, device=px.device) for _ in range(4))
    im = images_struct(dp.images)
    o = options(precision, **opt)
    phi, ex, ey, ez = out
    _check(lib.nebem_eval(ctypes.byref(dp.struct), ctypes.byref(im), _ptr(sigma), _ptr(px), _ptr(py),
                          _ptr(pz), m, _ptr(phi), _ptr(ex), _ptr(ey), _ptr(ez), ctypes.byref(o),
                          _stream(stream)))
    return out


class Session:
    """A geometry kept resident on the GPU: element records, factored
    influence matrix and the current surface charge densities."""

    def __init__(self, dp: DevicePanels, precision=FP64, stream=None, **opt):
        self.dp = dp
        self.n = dp.n
        self.device = dp.tensors["ox"].device
        self.options = options(precision, **opt)
        self.precision = precision
        im = images_struct(dp.images)
        h = ctypes.c_void_p()
        code = lib.nebem_session_create(ctypes.byref(dp.struct), ctypes.byref(im), ctypes.byref(self.options),
                                        _stream(stream), ctypes.byref(h))
        if code not in (NEBEM_OK, NEBEM_ENOCONV):
            _check(code)
        self.handle = h
        self.create_status = code

    def close(self):
        if getattr(self, "handle", None):
            lib.nebem_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sigma(self):
        """Copy of the current sigma (float64 device tensor)."""
        import torch
        view = _DeviceArray(lib.nebem_session_sigma(self.handle), self.n)
        torch.cuda.synchronize()
        return torch.as_tensor(view, device=self.dp.tensors["ox"].device).clone()

    def solve(self, b, stream=None):
        info = SolveInfo()
        code = lib.nebem_session_solve(self.handle, _ptr(b), ctypes.byref(info), _stream(stream))
        if code not in (NEBEM_OK, NEBEM_ENOCONV):
            _check(code)
        return code, info

    def condest(self, stream=None):
        """cond_1 estimate of the session's matrix (FP64 sessions)."""
        out = ctypes.c_double()
        _check(lib.nebem_session_condest(self.handle, ctypes.byref(out), _stream(stream)))
        return out.value

    def eval_points(self, px, py, pz, stream=None, out=None):
        import torch
        m = px.shape[0]
        if out is None:
            out = tuple(torch.empty(m, dtype=torch.float64, device=px.device) for _ in range(4))
        phi, ex, ey, ez = out
        _check(lib.nebem_session_eval(self.handle, _ptr(px), _ptr(py), _ptr(pz), m, _ptr(phi), _ptr(ex),
                                      _ptr(ey), _ptr(ez), _stream(stream)))
        return out

    def fastvol(self, values=None, grid=None, axes=None, stream=None):
        """Attach a FastVolume map that the session fills now and after
        every space-charge re-solve: grid = (origin, step, shape) or axes =
        (ax, ay, az) device tensors; values: (nodes, 4) float64 device
        tensor (allocated when None).  No grid and no axes: detach."""
        import torch
        if grid is None and axes is None:
            _check(lib.nebem_session_fastvol(self.handle, None, None, None, _stream(stream)))
            return None
        if grid is not None:
            g, nn = grid_struct(*grid), int(np.prod(grid[2]))
            a = None
        else:
            g, a = None, axes_struct(*axes)
            nn = int(axes[0].shape[0] * axes[1].shape[0] * axes[2].shape[0])
            self._fv_axes = axes  # kept alive while attached
        if values is None:
            values = torch.empty((nn, 4), dtype=torch.float64, device=self.device)
        _check(lib.nebem_session_fastvol(self.handle, ctypes.byref(g) if g is not None else None,
                                         ctypes.byref(a) if a is not None else None, _ptr(values),
                                         _stream(stream)))
        return values

    def eval_points_noalloc(self, px, py, pz, out, stream=None):
        """eval_points into caller-allocated outputs, with no device
        allocation by the library (its fixed scratch instead)."""
        phi, ex, ey, ez = out
        _check(lib.nebem_session_eval_noalloc(self.handle, _ptr(px), _ptr(py), _ptr(pz), px.shape[0], _ptr(phi),
                                              _ptr(ex), _ptr(ey), _ptr(ez), _stream(stream)))
        return out

    def spacecharge_step(self, qx, qy, qz, q, step_index, E=None, stream=None):
        """One explicit step of the dynamic space-charge loop, in place on
        (qx, qy, qz); returns the status (OK or ENOCONV)."""
        nq = qx.shape[0]
        ex = ey = ez = None
        if E is not None:
            ex, ey, ez = E
        code = lib.nebem_spacecharge_step(self.handle, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(q), nq,
                                          int(step_index), _ptr(ex), _ptr(ey), _ptr(ez), _stream(stream))
        if code not in (NEBEM_OK, NEBEM_ENOCONV):
            _check(code)
        return code

    def spacecharge_step_lines(self, qx, qy, qz, q, step_index, origin, step, shape, E=None, placement="centre",
                               stream=None):
        """The space-charge step with the charges reduced to line charges on
        the voxel grid (origin, step, shape) first; returns (status, lines)."""
        nq = qx.shape[0]
        ex = ey = ez = None
        if E is not None:
            ex, ey, ez = E
        g = grid_struct(origin, step, shape)
        nl = ctypes.c_int64()
        code = lib.nebem_spacecharge_step_lines(self.handle, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(q), nq,
                                                int(step_index), ctypes.byref(g), _PLACEMENT[placement],
                                                _ptr(ex), _ptr(ey), _ptr(ez),
                                                ctypes.byref(nl), _stream(stream))
        if code not in (NEBEM_OK, NEBEM_ENOCONV):
            _check(code)
        return code, nl.value


class _DeviceArray:
    """float64 device array at a raw address (array-interface view, used
    only to copy the data out)."""

    def __init__(self, ptr, n):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": "<f8", "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def _np_ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def server_default_options() -> ServerOptions:
    """The library's default server options (nebem_server_default_options)."""
    o = ServerOptions()
    lib.nebem_server_default_options(ctypes.byref(o))
    return o


class Server:
    """Continuous-batching evaluation service over resident sessions (host
    numpy arrays in and out; the arrays must stay alive until `wait`)."""

    def __init__(self, sessions, hbm_budget=None, batch_interactions=None, max_items=None,
                 large_interactions=None, max_large=None):
        o = ServerOptions()
        lib.nebem_server_default_options(ctypes.byref(o))
        if large_interactions is not None:
            o.large_interactions = float(large_interactions)
        if max_large is not None:
            o.max_large = int(max_large)
        if hbm_budget is not None:
            o.hbm_budget = int(hbm_budget)
        if batch_interactions is not None:
            o.batch_interactions = float(batch_interactions)
        if max_items is not None:
            o.max_items = int(max_items)
        self.sessions = list(sessions)
        arr = (ctypes.c_void_p * len(self.sessions))(*[s.handle for s in self.sessions])
        h = ctypes.c_void_p()
        _check(lib.nebem_server_create(arr, len(self.sessions), ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, geometry, pts, want=("phi", "ex", "ey", "ez")):
        """pts: (m, 3) float64.  Returns a ticket; results via wait()."""
        m = pts.shape[0]
        cols = [np.ascontiguousarray(pts[:, k], dtype=np.float64) for k in range(3)]
        outs = {k: (np.empty(m) if k in want else None) for k in ("phi", "ex", "ey", "ez")}
        t = ctypes.c_int64()
        _check(lib.nebem_server_submit(self.handle, int(geometry), *[_np_ptr(c) for c in cols], m,
                                       _np_ptr(outs["phi"]), _np_ptr(outs["ex"]), _np_ptr(outs["ey"]),
                                       _np_ptr(outs["ez"]), ctypes.byref(t)))
        self._keep[t.value] = (cols, outs)
        return t.value

    def wait(self, ticket):
        """Blocks until the request is done; returns (results dict, stats)."""
        st = RequestStats()
        code = lib.nebem_server_wait(self.handle, int(ticket), ctypes.byref(st))
        cols, outs = self._keep.pop(ticket)
        _check(code)
        return outs, st

    def counters(self):
        c = ServerCounters()
        _check(lib.nebem_server_stats(self.handle, ctypes.byref(c)))
        return c

    def close(self):
        if getattr(self, "handle", None):
            lib.nebem_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
