"""Synthetic MPGD-shaped boundary geometries made of flat panels.

A panel is either

* kind 0, a rectangle  { o + s*u + t*w : 0 <= s, t <= 1 }, or
* kind 1, a right triangle with the right angle at o,
  { o + s*u + t*w : s, t >= 0, s + t <= 1 },

with u perpendicular to w and unit normal n = (u x w)/|u x w|.  These are the
two element shapes of the paper (Sec. 2.1, rectangle and right-angled
triangle); a general triangle is split at the foot of the altitude on its
longest side into two right triangles.

Each panel carries a boundary condition: bc 0 = conductor held at potential
`value` (Dirichlet, Sec. 2), bc 1 = interface between two dielectrics with
relative permittivity `eps_pos` on the +n side and `eps_neg` on the -n side.

The geometries stand in for the paper's detector models (parallel plates,
Sec. 5.1; THGEM, Sec. 5.2), which are built there with Garfield++/neBEM
primitives that are not available here.  Everything is in SI units (metres,
volts).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CONDUCTOR = 0
DIELECTRIC = 1
RECT = 0
RTRI = 1


@dataclass
class Images:
    """Periodic (lattice) and mirror copies of the base cell.

    Translations t = n1*a1 + n2*a2 with |n1| <= n1max, |n2| <= n2max, visited
    with n1 in the outer and n2 in the inner loop.  Optional reflection planes
    x_k = mirror_pos[k] for every axis bit k set in `mirror_mask`; a copy
    reflected in a set of planes carries sigma times the product of their
    `mirror_parity` entries (+1 or -1).  Every combination of reflections is
    applied before every translation: copy = t + M(panel).
    """

    a1: np.ndarray = field(default_factory=lambda: np.zeros(3))
    a2: np.ndarray = field(default_factory=lambda: np.zeros(3))
    n1: int = 0
    n2: int = 0
    mirror_mask: int = 0
    mirror_pos: np.ndarray = field(default_factory=lambda: np.zeros(3))
    mirror_parity: np.ndarray = field(default_factory=lambda: np.ones(3, dtype=np.int32))

    @property
    def n_translations(self) -> int:
        return (2 * self.n1 + 1) * (2 * self.n2 + 1)

    @property
    def n_reflections(self) -> int:
        return 1 << bin(self.mirror_mask & 7).count("1")

    @property
    def count(self) -> int:
        return self.n_translations * self.n_reflections

    def translations(self) -> np.ndarray:
        out = []
        for i in range(-self.n1, self.n1 + 1):
            for j in range(-self.n2, self.n2 + 1):
                out.append(i * np.asarray(self.a1, float) + j * np.asarray(self.a2, float))
        return np.array(out, dtype=np.float64).reshape(-1, 3)


@dataclass
class Geometry:
    name: str
    kind: np.ndarray      # int32 [N]
    o: np.ndarray         # f64 [N,3]
    u: np.ndarray         # f64 [N,3]
    w: np.ndarray         # f64 [N,3]
    bc: np.ndarray        # int32 [N]
    value: np.ndarray     # f64 [N]
    eps_pos: np.ndarray   # f64 [N]
    eps_neg: np.ndarray   # f64 [N]
    images: Images
    box_lo: np.ndarray    # f64 [3], evaluation region (axis-aligned hull)
    box_hi: np.ndarray

    @property
    def n(self) -> int:
        return int(self.kind.shape[0])

    def soa(self) -> dict:
        """Contiguous structure-of-arrays view (the layout the C-ABI takes)."""
        c = np.ascontiguousarray
        return dict(
            kind=c(self.kind, dtype=np.int32),
            ox=c(self.o[:, 0]), oy=c(self.o[:, 1]), oz=c(self.o[:, 2]),
            ux=c(self.u[:, 0]), uy=c(self.u[:, 1]), uz=c(self.u[:, 2]),
            wx=c(self.w[:, 0]), wy=c(self.w[:, 1]), wz=c(self.w[:, 2]),
            bc=c(self.bc, dtype=np.int32), value=c(self.value),
            eps_pos=c(self.eps_pos), eps_neg=c(self.eps_neg),
        )

    def rhs(self) -> np.ndarray:
        """Known boundary values: V on conductors, 0 on dielectric interfaces."""
        return np.where(self.bc == CONDUCTOR, self.value, 0.0).astype(np.float64)

    def centroids(self) -> np.ndarray:
        f = np.where(self.kind == RECT, 0.5, 1.0 / 3.0)[:, None]
        return self.o + f * (self.u + self.w)

    def areas(self) -> np.ndarray:
        a = np.linalg.norm(np.cross(self.u, self.w), axis=1)
        return np.where(self.kind == RECT, a, 0.5 * a)

    def normals(self) -> np.ndarray:
        c = np.cross(self.u, self.w)
        return c / np.linalg.norm(c, axis=1)[:, None]

    def subset(self, idx) -> "Geometry":
        idx = np.asarray(idx)
        return Geometry(self.name + "[sub]", self.kind[idx], self.o[idx], self.u[idx],
                        self.w[idx], self.bc[idx], self.value[idx], self.eps_pos[idx],
                        self.eps_neg[idx], self.images, self.box_lo, self.box_hi)

    def with_images(self, images: Images) -> "Geometry":
        return Geometry(self.name, self.kind, self.o, self.u, self.w, self.bc, self.value,
                        self.eps_pos, self.eps_neg, images, self.box_lo, self.box_hi)


class GeometryBuilder:
    """Accumulates panels; general polygons are cut into rects/right triangles."""

    def __init__(self):
        self._kind, self._o, self._u, self._w = [], [], [], []
        self._bc, self._val, self._ep, self._en = [], [], [], []

    def __len__(self):
        return len(self._kind)

    def _add(self, kind, o, u, w, bc, value, eps_pos, eps_neg, normal):
        o = np.asarray(o, float)
        u = np.asarray(u, float)
        w = np.asarray(w, float)
        if normal is not None and np.dot(np.cross(u, w), normal) < 0:
            u, w = w, u  # the same rectangle / right triangle, opposite normal
        lu, lw = np.linalg.norm(u), np.linalg.norm(w)
        if lu <= 0 or lw <= 0:
            return
        # edge vectors must be perpendicular (up to rounding of the mesher);
        # remove the rounding residue so the panel is exactly a rectangle /
        # right triangle
        cos_uw = np.dot(w, u) / (lu * lw)
        if abs(cos_uw) > 1e-9:
            raise ValueError(f"panel edges not perpendicular (cos = {cos_uw:.3e})")
        w = w - np.dot(w, u) / (lu * lu) * u
        self._kind.append(kind)
        self._o.append(o)
        self._u.append(u)
        self._w.append(w)
        self._bc.append(bc)
        self._val.append(value)
        self._ep.append(eps_pos)
        self._en.append(eps_neg)

    def rect(self, o, u, w, bc=CONDUCTOR, value=0.0, eps_pos=1.0, eps_neg=1.0, normal=None):
        self._add(RECT, o, u, w, bc, value, eps_pos, eps_neg, normal)

    def right_tri(self, o, u, w, bc=CONDUCTOR, value=0.0, eps_pos=1.0, eps_neg=1.0, normal=None):
        self._add(RTRI, o, u, w, bc, value, eps_pos, eps_neg, normal)

    def triangle(self, a, b, c, normal=None, min_frac=1e-6, **bcargs):
        """General triangle -> two right triangles split at the altitude foot
        on the longest side."""
        pts = [np.asarray(p, float) for p in (a, b, c)]
        lens = [np.linalg.norm(pts[(k + 1) % 3] - pts[k]) for k in range(3)]
        k = int(np.argmax(lens))
        A, B, C = pts[k], pts[(k + 1) % 3], pts[(k + 2) % 3]
        if normal is None:
            normal = np.cross(B - A, C - A)
        AB = B - A
        t = np.dot(C - A, AB) / np.dot(AB, AB)
        F = A + t * AB
        if t > min_frac:
            self.right_tri(F, A - F, C - F, normal=normal, **bcargs)
        if t < 1.0 - min_frac:
            self.right_tri(F, B - F, C - F, normal=normal, **bcargs)

    def quad(self, p0, p1, p2, p3, normal=None, **bcargs):
        """Planar quadrilateral p0-p1-p2-p3: cut along the shorter diagonal."""
        p = [np.asarray(x, float) for x in (p0, p1, p2, p3)]
        if normal is None:
            normal = np.cross(p[2] - p[0], p[3] - p[1])
        if np.linalg.norm(p[2] - p[0]) <= np.linalg.norm(p[3] - p[1]):
            self.triangle(p[0], p[1], p[2], normal=normal, **bcargs)
            self.triangle(p[0], p[2], p[3], normal=normal, **bcargs)
        else:
            self.triangle(p[0], p[1], p[3], normal=normal, **bcargs)
            self.triangle(p[1], p[2], p[3], normal=normal, **bcargs)

    def trapezoid(self, a0, a1, b1, b0, normal=None, **bcargs):
        """Isosceles trapezoid with parallel sides a0-a1 and b0-b1 (same
        direction): one rectangle over the shorter side plus two right
        triangles."""
        a0, a1, b0, b1 = (np.asarray(x, float) for x in (a0, a1, b0, b1))
        if np.linalg.norm(a1 - a0) > np.linalg.norm(b1 - b0):
            a0, a1, b0, b1 = b0, b1, a0, a1
        d = (a1 - a0) / np.linalg.norm(a1 - a0)
        # feet of the short side's ends on the long side's line
        f0 = b0 + np.dot(a0 - b0, d) * d
        f1 = b0 + np.dot(a1 - b0, d) * d
        if normal is None:
            normal = np.cross(a1 - a0, b0 - a0)
        self.rect(f0, f1 - f0, a0 - f0, normal=normal, **bcargs)
        if np.dot(f0 - b0, d) > 1e-12 * np.linalg.norm(a1 - a0):
            self.right_tri(f0, b0 - f0, a0 - f0, normal=normal, **bcargs)
        if np.dot(b1 - f1, d) > 1e-12 * np.linalg.norm(a1 - a0):
            self.right_tri(f1, b1 - f1, a1 - f1, normal=normal, **bcargs)

    def build(self, name, images, box_lo, box_hi) -> Geometry:
        return Geometry(
            name=name,
            kind=np.array(self._kind, dtype=np.int32),
            o=np.array(self._o, dtype=np.float64).reshape(-1, 3),
            u=np.array(self._u, dtype=np.float64).reshape(-1, 3),
            w=np.array(self._w, dtype=np.float64).reshape(-1, 3),
            bc=np.array(self._bc, dtype=np.int32),
            value=np.array(self._val, dtype=np.float64),
            eps_pos=np.array(self._ep, dtype=np.float64),
            eps_neg=np.array(self._en, dtype=np.float64),
            images=images,
            box_lo=np.asarray(box_lo, float),
            box_hi=np.asarray(box_hi, float),
        )


# ---------------------------------------------------------------------------
# parallel plates (paper Sec. 5.1 shape; sizes of the 512-element benchmark)
# ---------------------------------------------------------------------------

def parallel_plates(n: int = 16, side: float = 1e-3, gap: float = 0.2e-3,
                    v_bottom: float = 0.0, v_top: float = 1.0) -> Geometry:
    """Two side x side plates at z = -gap/2 (v_bottom) and +gap/2 (v_top),
    each cut into n x n identical square panels with normal +z."""
    b = GeometryBuilder()
    h = side / n
    for z, v in ((-gap / 2, v_bottom), (gap / 2, v_top)):
        for i in range(n):
            for j in range(n):
                o = (-side / 2 + i * h, -side / 2 + j * h, z)
                b.rect(o, (h, 0, 0), (0, h, 0), bc=CONDUCTOR, value=v)
    return b.build("parallel_plates", Images(),
                   (-side / 2, -side / 2, -gap / 2), (side / 2, side / 2, gap / 2))


# ---------------------------------------------------------------------------
# helpers for perforated foils in a parallelogram (hexagonal-lattice) cell
# ---------------------------------------------------------------------------

def _cell_angles(center, corners, k):
    """k ray directions around `center`: uniform, with the ray nearest to each
    cell corner snapped onto that corner so every radial strip ends on one
    straight side of the cell."""
    ang = 2 * math.pi * np.arange(k) / k
    for c in corners:
        a = math.atan2(c[1] - center[1], c[0] - center[0]) % (2 * math.pi)
        d = np.abs((ang - a + math.pi) % (2 * math.pi) - math.pi)
        ang[int(np.argmin(d))] = a
    return np.sort(ang)


def _ray_to_cell(center, direction, corners):
    best = np.inf
    for i in range(4):
        p, q = corners[i], corners[(i + 1) % 4]
        e = q - p
        m = np.array([[direction[0], -e[0]], [direction[1], -e[1]]])
        rhs = p[:2] - center[:2]
        det = np.linalg.det(m)
        if abs(det) < 1e-30:
            continue
        lam, mu = np.linalg.solve(m, rhs)
        if lam > 0 and -1e-9 <= mu <= 1 + 1e-9:
            best = min(best, lam)
    return center[:2] + best * direction[:2]


def _face_with_hole(b, center, corners, angles, r_hole, nr, z, grade=1.3, normal=(0, 0, 1), **bc):
    """Planar cell face at height z with a polygonal hole of radius r_hole,
    meshed in radial strips (graded towards the hole)."""
    s = (np.arange(nr + 1) / nr) ** grade
    k = len(angles)
    inner, outer = [], []
    for a in angles:
        d = np.array([math.cos(a), math.sin(a)])
        inner.append(center[:2] + r_hole * d)
        outer.append(_ray_to_cell(center, d, corners))
    for i in range(k):
        j = (i + 1) % k
        for m in range(nr):
            p = []
            for (idx, sv) in ((i, s[m]), (j, s[m]), (j, s[m + 1]), (i, s[m + 1])):
                xy = inner[idx] + sv * (outer[idx] - inner[idx])
                p.append((xy[0], xy[1], z))
            b.quad(*p, normal=np.asarray(normal, float), **bc)


def _annulus(b, center, angles, r1, r2, nrad, z, normal=(0, 0, 1), **bc):
    k = len(angles)
    rs = np.linspace(r1, r2, nrad + 1)
    for i in range(k):
        j = (i + 1) % k
        ci, si = math.cos(angles[i]), math.sin(angles[i])
        cj, sj = math.cos(angles[j]), math.sin(angles[j])
        for m in range(nrad):
            ra, rb = rs[m], rs[m + 1]
            a0 = (center[0] + ra * ci, center[1] + ra * si, z)
            a1 = (center[0] + ra * cj, center[1] + ra * sj, z)
            b0 = (center[0] + rb * ci, center[1] + rb * si, z)
            b1 = (center[0] + rb * cj, center[1] + rb * sj, z)
            b.quad(a0, a1, b1, b0, normal=np.asarray(normal, float), **bc)


def _cylinder(b, center, angles, r, z1, z2, nz, inward=True, **bc):
    """Polygonal prism wall: each facet is an exact rectangle."""
    k = len(angles)
    zs = np.linspace(z1, z2, nz + 1)
    for i in range(k):
        j = (i + 1) % k
        p = np.array([center[0] + r * math.cos(angles[i]), center[1] + r * math.sin(angles[i])])
        q = np.array([center[0] + r * math.cos(angles[j]), center[1] + r * math.sin(angles[j])])
        mid = 0.5 * (p + q) - center[:2]
        nrm = np.array([-mid[0], -mid[1], 0.0]) if inward else np.array([mid[0], mid[1], 0.0])
        for m in range(nz):
            o = (p[0], p[1], zs[m])
            b.rect(o, (q[0] - p[0], q[1] - p[1], 0.0), (0.0, 0.0, zs[m + 1] - zs[m]),
                   normal=nrm, **bc)


def _cone(b, center, angles, r1, z1, r2, z2, nz, inward=True, **bc):
    """Frustum wall from (r1, z1) to (r2, z2); each isosceles-trapezoid facet
    is cut along its shorter diagonal (four right triangles)."""
    k = len(angles)
    ts = np.linspace(0.0, 1.0, nz + 1)
    for i in range(k):
        j = (i + 1) % k
        ci, si = math.cos(angles[i]), math.sin(angles[i])
        cj, sj = math.cos(angles[j]), math.sin(angles[j])
        cm, sm = math.cos(0.5 * (angles[i] + angles[j] + (2 * math.pi if j == 0 else 0))), \
            math.sin(0.5 * (angles[i] + angles[j] + (2 * math.pi if j == 0 else 0)))
        for m in range(nz):
            ra = r1 + (r2 - r1) * ts[m]
            rb = r1 + (r2 - r1) * ts[m + 1]
            za = z1 + (z2 - z1) * ts[m]
            zb = z1 + (z2 - z1) * ts[m + 1]
            a0 = (center[0] + ra * ci, center[1] + ra * si, za)
            a1 = (center[0] + ra * cj, center[1] + ra * sj, za)
            b0 = (center[0] + rb * ci, center[1] + rb * si, zb)
            b1 = (center[0] + rb * cj, center[1] + rb * sj, zb)
            # outward (away from the axis) radial direction, tilted by the slope
            dr, dz = rb - ra, zb - za
            radial = np.array([cm, sm, 0.0])
            nrm = radial * dz - np.array([0.0, 0.0, 1.0]) * dr
            if inward:
                nrm = -nrm
            b.quad(a0, a1, b1, b0, normal=nrm, **bc)


def _plane(b, origin, a1, a2, z, nd, **bc):
    """Whole-cell plane (drift cathode / anode): nd x nd sub-parallelograms,
    each two triangles (four right triangles)."""
    for i in range(nd):
        for j in range(nd):
            p0 = origin + (i / nd) * a1 + (j / nd) * a2
            p1 = p0 + a1 / nd
            p2 = p1 + a2 / nd
            p3 = p0 + a2 / nd
            pts = [(p[0], p[1], z) for p in (p0, p1, p2, p3)]
            b.quad(*pts, normal=np.array([0.0, 0.0, 1.0]), **bc)


def _hex_cell(pitch, origin_xy=(0.0, 0.0)):
    a1 = np.array([pitch, 0.0, 0.0])
    a2 = np.array([0.5 * pitch, 0.5 * math.sqrt(3.0) * pitch, 0.0])
    o = np.array([origin_xy[0], origin_xy[1], 0.0])
    corners = [o, o + a1, o + a1 + a2, o + a2]
    center = o + 0.5 * (a1 + a2)
    return a1, a2, o, corners, center


# ---------------------------------------------------------------------------
# single GEM unit cell (about 8 000 panels)
# ---------------------------------------------------------------------------

def gem_cell(k: int = 64, nr: int = 6, nz_kapton: int = 3, nz_cu: int = 1, nd: int = 8,
             n_images: int = 5) -> Geometry:
    """One hexagonal-lattice cell of a standard GEM: 50 um kapton (eps_r 3.5)
    clad with 5 um copper, 140 um pitch, one double-conical hole (70 um at
    the copper, 50 um in the middle), copper at -200 V (top) / +200 V
    (bottom), drift plane 3 mm above the top copper at -500 V.  Lattice
    copies +-n_images along both cell vectors."""
    um = 1e-6
    pitch = 140 * um
    t_k, t_cu = 50 * um, 5 * um
    r_out, r_mid = 35 * um, 25 * um
    a1, a2, o, corners, center = _hex_cell(pitch)
    ang = _cell_angles(center, corners, k)
    b = GeometryBuilder()
    z_kt, z_kb = t_k / 2, -t_k / 2
    z_ct, z_cb = z_kt + t_cu, z_kb - t_cu
    top = dict(bc=CONDUCTOR, value=-200.0)
    bot = dict(bc=CONDUCTOR, value=+200.0)
    for z, bcx in ((z_ct, top), (z_kt, top), (z_kb, bot), (z_cb, bot)):
        _face_with_hole(b, center, corners, ang, r_out, nr, z, **bcx)
    _cylinder(b, center, ang, r_out, z_kt, z_ct, nz_cu, **top)
    _cylinder(b, center, ang, r_out, z_cb, z_kb, nz_cu, **bot)
    # kapton wall: normal points into the gas (towards the axis), gas on +n
    diel = dict(bc=DIELECTRIC, value=0.0, eps_pos=1.0, eps_neg=3.5)
    _cone(b, center, ang, r_mid, 0.0, r_out, z_kt, nz_kapton, inward=True, **diel)
    _cone(b, center, ang, r_out, z_kb, r_mid, 0.0, nz_kapton, inward=True, **diel)
    z_drift = z_ct + 3e-3
    _plane(b, o, a1, a2, z_drift, nd, bc=CONDUCTOR, value=-500.0)
    imgs = Images(a1=a1, a2=a2, n1=n_images, n2=n_images)
    lo = np.array([0.0, 0.0, z_cb - 1e-3])
    hi = np.array([a1[0] + a2[0], a2[1], z_drift])
    return b.build("gem_cell", imgs, lo, hi)


# ---------------------------------------------------------------------------
# staggered double thick GEM (about 40 000 panels)
# ---------------------------------------------------------------------------

def _thgem_layer(b, z_bottom, v_bot, v_top, shift, k, nr, nrim, nz_fr4, nz_cu,
                 pitch, t_fr4, t_cu, r_hole, rim, eps_fr4):
    a1, a2, o, corners, center = _hex_cell(pitch, shift)
    ang = _cell_angles(center, corners, k)
    z0 = z_bottom                  # bottom of bottom copper
    z1 = z0 + t_cu                 # FR4 bottom face
    z2 = z1 + t_fr4                # FR4 top face
    z3 = z2 + t_cu                 # top of top copper
    r_cu = r_hole + rim
    top = dict(bc=CONDUCTOR, value=v_top)
    bot = dict(bc=CONDUCTOR, value=v_bot)
    for z, bcx in ((z3, top), (z2, top), (z1, bot), (z0, bot)):
        _face_with_hole(b, center, corners, ang, r_cu, nr, z, **bcx)
    _cylinder(b, center, ang, r_cu, z2, z3, nz_cu, **top)
    _cylinder(b, center, ang, r_cu, z0, z1, nz_cu, **bot)
    # exposed FR4 rims (gas above the top rim, below the bottom rim)
    _annulus(b, center, ang, r_hole, r_cu, nrim, z2, normal=(0, 0, 1),
             bc=DIELECTRIC, value=0.0, eps_pos=1.0, eps_neg=eps_fr4)
    _annulus(b, center, ang, r_hole, r_cu, nrim, z1, normal=(0, 0, -1),
             bc=DIELECTRIC, value=0.0, eps_pos=1.0, eps_neg=eps_fr4)
    _cylinder(b, center, ang, r_hole, z1, z2, nz_fr4, inward=True,
              bc=DIELECTRIC, value=0.0, eps_pos=1.0, eps_neg=eps_fr4)
    return z3


def thgem_double(k: int = 96, nr: int = 11, nrim: int = 2, nz_fr4: int = 12, nz_cu: int = 1,
                 nd: int = 16, n_images: int = 5) -> Geometry:
    """Two staggered THGEMs: 0.4 mm FR4 (eps_r 4.4) with 35 um copper, 0.4 mm
    holes with 50 um rims at 0.8 mm hexagonal pitch; the upper foil shifted
    by half a pitch along x; 2 mm transfer gap; anode 2 mm below the lower
    foil (0 V), drift cathode 9 mm above the upper foil (-5400 V); lower foil
    -800/-2000 V, upper foil -2400/-3600 V (bottom/top copper)."""
    mm = 1e-3
    pitch, t_fr4, t_cu = 0.8 * mm, 0.4 * mm, 0.035 * mm
    r_hole, rim = 0.2 * mm, 0.05 * mm
    b = GeometryBuilder()
    z_anode = 0.0
    z_l2 = z_anode + 2 * mm
    z_top2 = _thgem_layer(b, z_l2, -800.0, -2000.0, (0.0, 0.0), k, nr, nrim, nz_fr4, nz_cu,
                          pitch, t_fr4, t_cu, r_hole, rim, 4.4)
    z_l1 = z_top2 + 2 * mm
    z_top1 = _thgem_layer(b, z_l1, -2400.0, -3600.0, (0.5 * pitch, 0.0), k, nr, nrim, nz_fr4,
                          nz_cu, pitch, t_fr4, t_cu, r_hole, rim, 4.4)
    z_drift = z_top1 + 9 * mm
    a1, a2, o, corners, center = _hex_cell(pitch)
    _plane(b, o, a1, a2, z_anode, nd, bc=CONDUCTOR, value=0.0)
    _plane(b, o, a1, a2, z_drift, nd, bc=CONDUCTOR, value=-5400.0)
    imgs = Images(a1=a1, a2=a2, n1=n_images, n2=n_images)
    lo = np.array([0.0, 0.0, z_anode])
    hi = np.array([a1[0] + a2[0], a2[1], z_drift])
    return b.build("thgem_double", imgs, lo, hi)


def strip_cell(pitch: float = 100e-6, n_strips: int = 4, strip_w: float = 15e-6, gap: float = 128e-6,
               sub_u: int = 4, sub_w: int = 16, n_img: int = 5, split: int = 1):
    """Periodic readout-like cell for Adaptive Modelling: a pitch x pitch
    cell (copies +-n_img along x and y) with n_strips anode strips at z = 0
    (alternating +-50 V) and a mesh plane at z = gap (-400 V).  Each strip
    is `split` primitives along its length and the plane split x split
    primitives; every primitive (a flat rectangle) is cut into sub_u x sub_w
    rectangular elements.  Returns (elements, primitives, elem_prim)."""
    eb, pb = GeometryBuilder(), GeometryBuilder()
    emap = []
    prims = []
    dx = pitch / n_strips
    for s in range(n_strips):
        x0 = s * dx + 0.5 * (dx - strip_w)
        for t in range(split):
            prims.append(((x0, t * pitch / split, 0.0), (strip_w, 0.0, 0.0), (0.0, pitch / split, 0.0),
                          50.0 * (-1) ** s))
    for a in range(split):
        for b in range(split):
            prims.append(((a * pitch / split, b * pitch / split, gap), (pitch / split, 0.0, 0.0),
                          (0.0, pitch / split, 0.0), -400.0))
    for p, (o, u, w, v) in enumerate(prims):
        pb.rect(o, u, w, bc=CONDUCTOR, value=v)
        for a in range(sub_u):
            for b in range(sub_w):
                oo = tuple(o[k] + a * u[k] / sub_u + b * w[k] / sub_w for k in range(3))
                eb.rect(oo, tuple(c / sub_u for c in u), tuple(c / sub_w for c in w), bc=CONDUCTOR, value=v)
                emap.append(p)
    im = Images(a1=np.array([pitch, 0.0, 0.0]), a2=np.array([0.0, pitch, 0.0]), n1=n_img, n2=n_img)
    box_lo, box_hi = (0.0, 0.0, 5e-6), (pitch, pitch, gap - 5e-6)
    return (eb.build("strip_cell", im, box_lo, box_hi), pb.build("strip_cell_primitives", im, box_lo, box_hi),
            np.asarray(emap, dtype=np.int32))
