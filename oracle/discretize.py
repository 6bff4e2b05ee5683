"""Visibility texture and truncated-Gaussian approximation (FP64 test infrastructure).

* Visibility (Section 3, last paragraph): a texel is marked visible when it
  lies inside the cascade polygon.  Rays need all four corners of every cell
  they may hit, so the reading here is: texture cell ``(i, j)`` spans texel
  centres ``i..i+1, j..j+1``; a cell is active when its closed rectangle
  meets the closed polygon (separating-axis test); a texel is visible when
  any of its (up to four) incident cells is active.  Invisible texels hold
  ``-inf``.
* Eq. 1: ``w_j(p) = exp(-(|p_j - p| / c_j)^2 / (2 sigma^2)) - exp(-k^2 / 2)``
  with the paper's ``k = 3.5``; here ``sigma`` may differ per leaf and ``k``
  is a parameter.  Leaf ``j`` influences ``p`` iff ``w_j(p) > 0``.
* Eq. 2: ``v(p) = sum_j w_j v_j / sum_j w_j`` over the influencing leaves.
* Another basis in Eq. 2's place of Eq. 1 (the two-step design admits any
  reconstruction, Section 1 and Section 7): Wendland's compactly supported
  C2 function ``phi(u) = (1 - u)^4 (4u + 1)`` for ``u < 1``, 0 beyond, with
  ``u = |p_j - p| / (k sigma_j c_j)`` -- the same support radius as the
  truncated Gaussian, so the same leaves influence the same points.
* A visible texel whose centre lies outside the domain is evaluated at the
  centre clamped into the domain (reading; the paper is silent).

Pinned by ``tests/test_oracle_discretize.py`` (both bases where it applies,
and ``tests/test_oracle_basis.py`` for the Wendland function: its integral
over the plane, its value and derivatives at 0 and at the support edge, the
derivative in sigma by finite differences): brute force over all leaves
equals the range-query sum to 1e-12; a tilted plane on a uniform grid is
reproduced exactly (symmetric neighbourhoods cancel first moments); the
result stays within the influencing values; the truncated sum stays within
the stated bound of the untruncated Gaussian sum; the mask against polygon
clipping by rectangles.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
from scipy.spatial import cKDTree

from . import build as _build


# ---------------------------------------------------------------- visibility

def cell_active_sat(cas, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Separating-axis test of texture cells ``(i, j)`` against the closed cascade polygon."""
    poly = np.asarray(cas.poly, np.float64)
    i = np.asarray(i, np.float64)
    j = np.asarray(j, np.float64)
    if len(poly) == 0:
        return np.zeros(i.shape, dtype=bool)
    xa, xb = cas.x0 + i * cas.hx, cas.x0 + (i + 1.0) * cas.hx
    ya, yb = cas.y0 + j * cas.hy, cas.y0 + (j + 1.0) * cas.hy
    sep = (xb < poly[:, 0].min()) | (xa > poly[:, 0].max()) | (yb < poly[:, 1].min()) | (ya > poly[:, 1].max())
    m = len(poly)
    for a in range(m if m > 2 else m - 1):
        p, q = poly[a], poly[(a + 1) % m]
        nx, ny = -(q[1] - p[1]), q[0] - p[0]
        proj_poly = poly[:, 0] * nx + poly[:, 1] * ny
        lo_p, hi_p = proj_poly.min(), proj_poly.max()
        c = np.stack([xa * nx + ya * ny, xb * nx + ya * ny, xa * nx + yb * ny, xb * nx + yb * ny])
        sep |= (c.max(axis=0) < lo_p) | (c.min(axis=0) > hi_p)
    return ~sep


def visibility(cas) -> np.ndarray:
    """Boolean ``[N][N]`` texel visibility (row = j)."""
    N = cas.n
    jj, ii = np.meshgrid(np.arange(N - 1), np.arange(N - 1), indexing="ij")
    act = cell_active_sat(cas, ii, jj)
    vis = np.zeros((N, N), dtype=bool)
    vis[:-1, :-1] |= act
    vis[:-1, 1:] |= act
    vis[1:, :-1] |= act
    vis[1:, 1:] |= act
    return vis


def texel_centres(cas, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    return np.stack([cas.x0 + np.asarray(i, np.float64) * cas.hx,
                     cas.y0 + np.asarray(j, np.float64) * cas.hy], axis=-1)


# ---------------------------------------------------------------- Eq. 1 / Eq. 2

BASES = ("gaussian", "wendland")


def basis_weight(q: np.ndarray, cutoff: float, basis: str = "gaussian") -> np.ndarray:
    """Weight at ``q = r / (sigma c)`` (unclipped for the Gaussian: Eq. 1 may go negative)."""
    if basis == "gaussian":
        return np.exp(-0.5 * q * q) - math.exp(-0.5 * cutoff * cutoff)
    if basis == "wendland":
        u = q / cutoff
        return np.where(u < 1.0, (1.0 - u) ** 4 * (4.0 * u + 1.0), 0.0)
    raise ValueError(f"unknown basis {basis!r}")


def basis_dweight_dsigma(q: np.ndarray, sigma: np.ndarray, cutoff: float, basis: str = "gaussian") -> np.ndarray:
    """``d w / d sigma`` at ``q = r / (sigma c)`` (q itself scales as 1 / sigma)."""
    if basis == "gaussian":
        return np.exp(-0.5 * q * q) * q * q / sigma
    if basis == "wendland":
        # w = (1 - u)^4 (4u + 1): dw/du = -20 u (1 - u)^3, du/dsigma = -u / sigma
        u = q / cutoff
        return np.where(u < 1.0, 20.0 * u * u * (1.0 - u) ** 3 / sigma, 0.0)
    raise ValueError(f"unknown basis {basis!r}")


def weights(p: np.ndarray, xj, yj, cj, sj, cutoff: float, basis: str = "gaussian") -> np.ndarray:
    """Eq. 1 (or the other basis) for points ``p (m, 2)`` against leaves ``j`` (broadcast ``(m, L)``),
    clipped at 0."""
    r = np.hypot(np.asarray(xj, np.float64)[None, :] - p[:, 0:1], np.asarray(yj, np.float64)[None, :] - p[:, 1:2])
    q = r / (np.asarray(sj, np.float64)[None, :] * np.asarray(cj, np.float64)[None, :])
    w = basis_weight(q, cutoff, basis)
    return np.where(w > 0.0, w, 0.0)


def clamp_to_domain(p: np.ndarray, dom) -> np.ndarray:
    return np.stack([np.clip(p[:, 0], dom.x0, dom.x1), np.clip(p[:, 1], dom.y0, dom.y1)], axis=-1)


def rbf_bruteforce(p: np.ndarray, leaves: dict, cutoff: float, chunk: int = 2048, basis: str = "gaussian") -> tuple:
    """Eq. 2 at points ``p`` summing over every leaf. Returns ``(value, sum_w)``."""
    out_v = np.empty(len(p))
    out_s = np.empty(len(p))
    for a in range(0, len(p), chunk):
        w = weights(p[a:a + chunk], leaves["x"], leaves["y"], leaves["c"], leaves["sigma"], cutoff, basis)
        s0 = w.sum(axis=1)
        out_v[a:a + chunk] = (w @ np.asarray(leaves["v"], np.float64)) / s0
        out_s[a:a + chunk] = s0
    return out_v, out_s


class RBFField:
    """Eq. 2 by range queries: one k-d tree per cell size, radius = cutoff * max(sigma) * c."""

    def __init__(self, leaves: dict, cutoff: float, basis: str = "gaussian"):
        if basis not in BASES:
            raise ValueError(f"unknown basis {basis!r}")
        self.L = {k: np.asarray(leaves[k], np.float64) for k in ("x", "y", "c", "v", "sigma")}
        self.cutoff = cutoff
        self.basis = basis
        self.groups = []
        for c in np.unique(self.L["c"]):
            idx = np.nonzero(self.L["c"] == c)[0]
            tree = cKDTree(np.stack([self.L["x"][idx], self.L["y"][idx]], axis=1))
            radius = cutoff * float(self.L["sigma"][idx].max()) * float(c)
            self.groups.append((idx, tree, radius))

    def candidates(self, p: np.ndarray) -> tuple:
        """Flat ``(point_index, leaf_index)`` pairs of every leaf within its group radius."""
        pi, lj = [], []
        for idx, tree, radius in self.groups:
            hits = tree.query_ball_point(p, radius)
            lens = np.fromiter((len(h) for h in hits), dtype=np.int64, count=len(hits))
            if lens.sum() == 0:
                continue
            pi.append(np.repeat(np.arange(len(p)), lens))
            lj.append(idx[np.concatenate([np.asarray(h, np.int64) for h in hits if h])])
        if not pi:
            return np.zeros(0, np.int64), np.zeros(0, np.int64)
        return np.concatenate(pi), np.concatenate(lj)

    def evaluate(self, p: np.ndarray, return_terms: bool = False):
        """``(value, sum_w)`` at points ``p``; optionally the flat ``(point, leaf, w)`` terms."""
        pi, lj = self.candidates(p)
        L = self.L
        r = np.hypot(L["x"][lj] - p[pi, 0], L["y"][lj] - p[pi, 1])
        q = r / (L["sigma"][lj] * L["c"][lj])
        w = basis_weight(q, self.cutoff, self.basis)
        keep = w > 0.0
        pi, lj, w = pi[keep], lj[keep], w[keep]
        s0 = np.bincount(pi, weights=w, minlength=len(p))
        s1 = np.bincount(pi, weights=w * L["v"][lj], minlength=len(p))
        with np.errstate(invalid="ignore", divide="ignore"):
            val = s1 / s0
        return (val, s0, (pi, lj, w)) if return_terms else (val, s0)


def discretize(cas, leaves: dict, dom, cutoff: float, field: RBFField = None, basis: str = "gaussian") -> np.ndarray:
    """FP64 cascade texture ``[N][N]``: Eq. 2 at visible texels, ``-inf`` elsewhere."""
    N = cas.n
    vis = visibility(cas)
    tex = np.full((N, N), -np.inf)
    jj, ii = np.nonzero(vis)
    if len(jj) == 0:
        return tex
    p = clamp_to_domain(texel_centres(cas, ii, jj), dom)
    if field is None:
        field = RBFField(leaves, cutoff, basis)
    tex[jj, ii] = field.evaluate(p)[0]
    return tex


# ---------------------------------------------------------------- plain-C form for full-size scenes

_clib = None


def _c_lib():
    global _clib
    if _clib is None:
        path = _build.library_path("rbf_oracle")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SOURCES["rbf_oracle"]):
            _build.build(force=False)
        lib = ctypes.CDLL(path)
        P, I64, F64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        lib.oracle_rbf_eval.argtypes = [I64, P, P, P, P, P, F64, I32, I64, P, P, P, P, I32]
        lib.oracle_rbf_eval.restype = I32
        lib.oracle_rbf_adjoint.argtypes = [I64, P, P, P, P, P, F64, I32, I64, P, P, P, P, P]
        lib.oracle_rbf_adjoint.restype = I32
        _clib = lib
    return _clib


def _leaf_arrays(leaves: dict):
    return [np.ascontiguousarray(leaves[k], np.float64) for k in ("x", "y", "c", "v", "sigma")]


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def rbf_evaluate_c(leaves: dict, cutoff: float, p: np.ndarray, basis: str = "gaussian", threads: int = 1) -> tuple:
    """Eq. 2 at points ``p (m, 2)`` (already clamped) by the plain-C form in ``oracle/c/rbf_oracle.c``:
    ``(value, sum_w)``, the same definition as ``RBFField.evaluate`` (every leaf with w > 0)."""
    if basis not in BASES:
        raise ValueError(f"unknown basis {basis!r}")
    arrs = _leaf_arrays(leaves)
    p = np.asarray(p, np.float64)
    px, py = np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1])
    val, s0 = np.empty(len(p)), np.empty(len(p))
    rc = _c_lib().oracle_rbf_eval(len(arrs[0]), *(_p(a) for a in arrs), float(cutoff), BASES.index(basis), len(p),
                                  _p(px), _p(py), _p(val), _p(s0), int(threads))
    if rc != 0:
        raise ValueError("oracle_rbf_eval rejected its arguments")
    return val, s0


def discretize_c(cas, leaves: dict, dom, cutoff: float, basis: str = "gaussian", threads: int = 1) -> np.ndarray:
    """``discretize`` with Eq. 2 evaluated by the plain-C form (full-size scenes)."""
    N = cas.n
    vis = visibility(cas)
    tex = np.full((N, N), -np.inf)
    jj, ii = np.nonzero(vis)
    if len(jj) == 0:
        return tex
    p = clamp_to_domain(texel_centres(cas, ii, jj), dom)
    tex[jj, ii] = rbf_evaluate_c(leaves, cutoff, p, basis, threads)[0]
    return tex
