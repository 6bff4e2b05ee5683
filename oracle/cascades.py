"""Cascade fitting (Section 3), FP64 test infrastructure.

Steps, in the paper's order:

1. Intersect the view frustum with the heightfield's bounding box.  Here the
   intersection is a convex polyhedron given by 11 half-spaces (6 box faces,
   the near plane, 4 side planes; the far plane is at infinity) and its
   vertices are found by brute force: every triple of planes is solved and
   the points satisfying all half-spaces are kept.
2. Project those vertices orthographically to the ground plane and take the
   convex hull (the potentially visible area).
3. Along the normalised 2-D projection ``v`` of the view vector, take the
   smallest and largest hull offsets ``n`` and ``f`` with the offset
   ``d(p) = (p - camera_xy) . v`` (reading: offsets measured from the camera).
4. Split the range.  The paper gives ``n (f/n)^(1/3)`` and ``n (f/n)^(2/3)``
   for three cascades; for ``K`` cascades this uses the practical split
   ``s_k = lam * n' (f/n')^(k/K) + (1 - lam) * (n + (f - n) k / K)``, which
   is the paper's formula at ``lam = 1, K = 3`` (reading).  ``n'`` is
   ``max(n, znear, c_min)`` because ``n`` may be zero or negative when the
   camera stands inside the box; when ``f <= n'`` the logarithmic term falls
   back to the uniform one.
5. Clip the hull against each cascade's near and far planes: the first near
   plane is ``n``, every other near plane is the previous split; the last far
   plane is ``f``, every other far plane is its split pushed out by
   ``delta_k = omega * (s_k - near_k)`` so that neighbours overlap (the
   paper's "small distance" is unspecified; ``omega`` is a reading).
6. Take each clipped polygon's axis-aligned box, widen its origin down to the
   ``c_min`` lattice and its extents up to an even multiple of ``c_min``,
   and map it onto the ``N x N`` texture so that the four box corners sit on
   the four corner texel centres: texel ``(i, j)`` is at
   ``(x0 + i hx, y0 + j hy)`` with ``hx = ext_x / (N - 1)`` (reading: the
   texels may be anisotropic; the paper asks for the largest used area).

A second fit keeps texel lattices fixed in the world between frames (for
reusing texels, not in the paper): each axis takes the smallest texel
spacing ``h = c_min 2^(e/4)`` (an integer ``e``, quarter octaves of the
smallest cell) for which the lattice origin, the largest multiple of ``h``
from the domain origin at or below the box, puts the last texel centre at
or beyond the box.  Two frames that pick the same ``h`` share the lattice
(their origins differ by whole texels).

Pinned by ``tests/test_oracle_cascades.py``: the three-cascade logarithmic
splits in closed form, a flat box whose visible area is the closed-form
trapezoid of the four corner rays, coverage of the hull by the cascades,
overlap widths, lattice and corner-alignment invariants.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List

import numpy as np

from .camera import basis

SNAP_TOL = 1e-9
MAX_POLY = 32


@dataclasses.dataclass
class Cascade:
    near: float
    far: float
    split: float
    origin: np.ndarray  # camera xy, origin of the offset d
    vhat: np.ndarray    # unit 2-D view direction
    x0: float
    y0: float
    hx: float
    hy: float
    n: int
    poly: np.ndarray    # (m, 2) counter-clockwise convex polygon, m may be 0

    def offset(self, p: np.ndarray) -> np.ndarray:
        return (p[..., 0] - self.origin[0]) * self.vhat[0] + (p[..., 1] - self.origin[1]) * self.vhat[1]


def _halfspaces(cam, dom) -> tuple:
    """Rows ``(a, h)`` meaning ``a . p >= h`` for the box and the frustum."""
    fwd, right, up = basis(cam)
    o = np.asarray(cam.pos, np.float64)
    ty = math.tan(0.5 * cam.vfov)
    tx = ty * cam.width / cam.height
    rows = [((1, 0, 0), dom.x0), ((-1, 0, 0), -dom.x1), ((0, 1, 0), dom.y0), ((0, -1, 0), -dom.y1),
            ((0, 0, 1), dom.zmin), ((0, 0, -1), -dom.zmax)]
    A = [np.array(a, np.float64) for a, _ in rows]
    H = [float(h) for _, h in rows]
    # near plane: fwd . (p - o) >= znear; sides: tx (fwd . q) -/+ right . q >= 0 etc.
    for a in (fwd, tx * fwd - right, tx * fwd + right, ty * fwd - up, ty * fwd + up):
        A.append(a / np.linalg.norm(a))
    H.append(float(A[6] @ o) + cam.znear)
    for k in range(7, 11):
        H.append(float(A[k] @ o))
    return np.array(A), np.array(H)


def frustum_box_vertices(cam, dom) -> np.ndarray:
    """Vertices ``(m, 3)`` of view frustum intersected with the box (brute force over plane triples)."""
    A, H = _halfspaces(cam, dom)
    scale = max(1.0, abs(dom.x0), abs(dom.x1), abs(dom.y0), abs(dom.y1), abs(dom.zmin), abs(dom.zmax),
                *[abs(c) for c in cam.pos])
    tol = 1e-9 * scale
    pts = []
    for i, j, k in itertools.combinations(range(len(A)), 3):
        M = A[[i, j, k]]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        p = np.linalg.solve(M, H[[i, j, k]])
        if np.all(A @ p >= H - tol):
            pts.append(p)
    return np.array(pts).reshape(-1, 3)


def convex_hull(points: np.ndarray) -> np.ndarray:
    """Counter-clockwise hull (Andrew's monotone chain), collinear points dropped."""
    pts = sorted(set(map(tuple, np.asarray(points, np.float64))))
    if len(pts) <= 2:
        return np.array(pts).reshape(-1, 2)

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return np.array(lower[:-1] + upper[:-1])


def clip_halfplane(poly: np.ndarray, g) -> np.ndarray:
    """Part of a convex polygon where the affine function ``g`` is ``>= 0``."""
    out = []
    m = len(poly)
    for a in range(m):
        p, q = poly[a], poly[(a + 1) % m]
        gp, gq = g(p), g(q)
        if gp >= 0:
            out.append(p)
        if (gp >= 0) != (gq >= 0) and m > 1:
            s = gp / (gp - gq)
            out.append(p + s * (q - p))
    if not out:
        return np.zeros((0, 2))
    # drop consecutive duplicates
    res = [out[0]]
    for p in out[1:]:
        if not np.array_equal(p, res[-1]):
            res.append(p)
    if len(res) > 1 and np.array_equal(res[0], res[-1]):
        res.pop()
    return np.array(res)


def split_distances(n: float, f: float, K: int, lam: float, znear: float, c_min: float) -> List[float]:
    """Practical split distances ``s_1 .. s_{K-1}``."""
    nprime = max(n, znear, c_min)
    out = []
    for k in range(1, K):
        uni = n + (f - n) * k / K
        log = nprime * (f / nprime) ** (k / K) if f > nprime else uni
        out.append(lam * log + (1.0 - lam) * uni)
    return out


def snap_axis(lo: float, hi: float, origin: float, c_min: float, N: int) -> tuple:
    """Stable fit of one axis: origin on the ``c_min`` lattice, extent an even multiple of it."""
    x0 = origin + math.floor((lo - origin) / c_min + SNAP_TOL) * c_min
    ext = max(1, math.ceil((hi - x0) / (2.0 * c_min) - SNAP_TOL)) * 2.0 * c_min
    return x0, ext / (N - 1)


QUARTER_OCTAVES = (1.0, 2.0 ** 0.25, 2.0 ** 0.5, 2.0 ** 0.75)


def snap_axis_aligned(lo: float, hi: float, origin: float, c_min: float, N: int) -> tuple:
    """Fixed-lattice fit of one axis: spacing on the quarter-octave ladder of ``c_min``, origin a
    multiple of the spacing; the smallest spacing that covers ``[lo, hi]``."""
    need = max(hi - lo, 0.0) / (N - 1)
    e = math.floor(4.0 * math.log2(need / c_min)) - 1 if need > 0 else -64
    while True:
        q, r = divmod(e, 4)
        h = math.ldexp(c_min * QUARTER_OCTAVES[r], q)
        x0 = origin + math.floor((lo - origin) / h + SNAP_TOL) * h
        if x0 + (N - 1) * h >= hi - SNAP_TOL * h:
            return x0, h
        e += 1


def fit_cascades(cam, dom, K: int, N: int, lam: float, omega: float, c_min: float,
                 aligned: bool = False) -> List[Cascade]:
    if K < 1 or N < 2 or N & (N - 1):
        raise ValueError("need K >= 1 and N a power of two >= 2")
    fwd, _, _ = basis(cam)
    vxy = np.array([fwd[0], fwd[1]])
    if np.linalg.norm(vxy) < 1e-12:
        raise ValueError("view vector has no horizontal component")
    vhat = vxy / np.linalg.norm(vxy)
    origin = np.array([cam.pos[0], cam.pos[1]], np.float64)
    verts = frustum_box_vertices(cam, dom)
    hull = convex_hull(verts[:, :2]) if len(verts) else np.zeros((0, 2))
    empty = Cascade(0.0, 0.0, 0.0, origin, vhat, dom.x0, dom.y0, 2.0 * c_min / (N - 1),
                    2.0 * c_min / (N - 1), N, np.zeros((0, 2)))
    if len(hull) == 0:
        return [dataclasses.replace(empty) for _ in range(K)]
    d = (hull[:, 0] - origin[0]) * vhat[0] + (hull[:, 1] - origin[1]) * vhat[1]
    n, f = float(d.min()), float(d.max())
    s = split_distances(n, f, K, lam, cam.znear, c_min)
    out = []
    for k in range(K):
        near = n if k == 0 else s[k - 1]
        split = s[k] if k < K - 1 else f
        far = split + omega * (split - near) if k < K - 1 else f

        def g_near(p, near=near):
            return (p[0] - origin[0]) * vhat[0] + (p[1] - origin[1]) * vhat[1] - near

        def g_far(p, far=far):
            return far - ((p[0] - origin[0]) * vhat[0] + (p[1] - origin[1]) * vhat[1])

        poly = clip_halfplane(clip_halfplane(hull, g_near), g_far)
        if len(poly) > MAX_POLY:
            raise ValueError("cascade polygon has too many vertices")
        if len(poly) == 0:
            out.append(dataclasses.replace(empty, near=near, far=far, split=split))
            continue
        snap = snap_axis_aligned if aligned else snap_axis
        x0, hx = snap(poly[:, 0].min(), poly[:, 0].max(), dom.x0, c_min, N)
        y0, hy = snap(poly[:, 1].min(), poly[:, 1].max(), dom.y0, c_min, N)
        out.append(Cascade(near, far, split, origin.copy(), vhat.copy(), x0, y0, hx, hy, N, poly))
    return out
