"""Hand-derived gradients of the hit depth (FP64 test infrastructure).

The paper has no backward pass; these are the derivatives of the forward
definitions in this oracle:

* Hit depth w.r.t. texel heights.  At a patch root ``f(t*) = 0`` with
  ``f(t) = z(t) - B(u(t), v(t))`` and ``B = sum_c h_c phi_c(u, v)``, the
  implicit function theorem gives ``dt*/dh_c = phi_c(u*, v*) / f'(t*)``
  with ``phi = ((1-u)(1-v), u(1-v), (1-u)v, uv)`` for corners
  ``(i, j), (i+1, j), (i, j+1), (i+1, j+1)``.  A hit at the start of a
  cascade segment sits on a boundary that does not depend on heights (zero).
  In overlaps the depth is ``(1 - a) t_near + a t_far`` with ``a`` a function
  of ``t_A``; the chain factors ``d depth / d t_A`` and ``d depth / d t_B``
  come from the C walk.
* Eq. 2 w.r.t. leaf values and widths: ``dv_s/dv_j = w_j / S0`` and
  ``dv_s/dsigma_j = (v_j - v_s) / S0 * dw_j/dsigma_j`` with
  ``dw_j/dsigma_j = exp(-q^2/2) q^2 / sigma_j``, ``q = r / (sigma_j c_j)``;
  the truncation constant does not depend on sigma.  With the Wendland basis
  ``w = (1 - u)^4 (4u + 1)``, ``u = q / k``: ``dw_j/dsigma_j = 20 u^2 (1 - u)^3 / sigma_j``.
* Central finite differences of the whole oracle pipeline for the checks.

Pinned by ``tests/test_oracle_adjoint.py``: finite differences, the
closed-form ``d depth / d C = 1 / d_z`` of a flat field, zero width gradient
on a constant field and partition of unity.
"""
from __future__ import annotations

import math

import numpy as np

from . import discretize as _disc
from .discretize import basis_dweight_dsigma, clamp_to_domain, texel_centres


def texel_gradients(res: dict, grad_depth: np.ndarray, K: int, N: int) -> np.ndarray:
    """``d loss / d tex`` (``[K][N][N]``) from ``d loss / d depth`` per cast ray."""
    g = np.zeros((K, N, N))
    gd = np.asarray(grad_depth, np.float64).ravel()
    for x in (0, 1):
        k, i, j, start = (res["rec"][:, 4 * x + a] for a in range(4))
        u, v, fp = res["val"][:, 4 * x + 1], res["val"][:, 4 * x + 2], res["val"][:, 4 * x + 3]
        sel = (k >= 0) & (start == 0) & (fp < 0.0) & (gd != 0.0)
        s = gd[sel] * res["coef"][sel, x] / fp[sel]
        k, i, j, u, v = k[sel], i[sel], j[sel], u[sel], v[sel]
        np.add.at(g, (k, j, i), s * (1 - u) * (1 - v))
        np.add.at(g, (k, j, i + 1), s * u * (1 - v))
        np.add.at(g, (k, j + 1, i), s * (1 - u) * v)
        np.add.at(g, (k, j + 1, i + 1), s * u * v)
    return g


def leaf_gradients(cascades, field, dom, gtex: np.ndarray) -> tuple:
    """``(d loss / d v, d loss / d sigma)`` per leaf from texel gradients (Eq. 2 adjoint)."""
    L = field.L
    gv = np.zeros(len(L["x"]))
    gs = np.zeros(len(L["x"]))
    for k, cas in enumerate(cascades):
        jj, ii = np.nonzero(gtex[k] != 0.0)
        if len(jj) == 0:
            continue
        gsx = gtex[k][jj, ii]
        p = clamp_to_domain(texel_centres(cas, ii, jj), dom)
        val, s0, (pi, lj, w) = field.evaluate(p, return_terms=True)
        gv += np.bincount(lj, weights=gsx[pi] * w / s0[pi], minlength=len(gv))
        r = np.hypot(L["x"][lj] - p[pi, 0], L["y"][lj] - p[pi, 1])
        q = r / (L["sigma"][lj] * L["c"][lj])
        dw = basis_dweight_dsigma(q, L["sigma"][lj], field.cutoff, getattr(field, "basis", "gaussian"))
        gs += np.bincount(lj, weights=gsx[pi] * (L["v"][lj] - val[pi]) / s0[pi] * dw, minlength=len(gs))
    return gv, gs


def l2_loss(depth: np.ndarray, target: np.ndarray) -> tuple:
    """``sum (depth - target)^2`` over pixels where both hit, and its gradient."""
    both = np.isfinite(depth) & np.isfinite(target)
    diff = np.where(both, np.where(both, depth, 0.0) - np.where(both, target, 0.0), 0.0)
    return float((diff * diff).sum()), 2.0 * diff


def cutoff_weight(cutoff: float) -> float:
    return math.exp(-0.5 * cutoff * cutoff)


def leaf_gradients_c(cascades, leaves: dict, cutoff: float, dom, gtex: np.ndarray, basis: str = "gaussian") -> tuple:
    """``leaf_gradients`` by the plain-C form of Eq. 2's adjoint (``oracle/c/rbf_oracle.c``), for full-size
    scenes: the same sums over every texel with a non-zero gradient and every leaf with w > 0."""
    arrs = _disc._leaf_arrays(leaves)
    n = len(arrs[0])
    gv, gs = np.zeros(n), np.zeros(n)
    lib = _disc._c_lib()
    for k, cas in enumerate(cascades):
        jj, ii = np.nonzero(gtex[k] != 0.0)
        if len(jj) == 0:
            continue
        p = clamp_to_domain(texel_centres(cas, ii, jj), dom)
        px, py = np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1])
        g = np.ascontiguousarray(gtex[k][jj, ii], np.float64)
        rc = lib.oracle_rbf_adjoint(n, *(_disc._p(a) for a in arrs), float(cutoff), _disc.BASES.index(basis), len(p),
                                    _disc._p(px), _disc._p(py), _disc._p(g), _disc._p(gv), _disc._p(gs))
        if rc != 0:
            raise ValueError("oracle_rbf_adjoint rejected its arguments")
    return gv, gs
