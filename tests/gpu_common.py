"""Shared pieces of the GPU parity tests: device inputs and comparison rules.

Tolerances (the stated parity bar):
* texel heights: |dv| <= 1e-5 * max(|v_oracle|, V), V = max |leaf value|;
* hit depth: |dt| <= 1e-4 * scene extent;
* hit cell: mismatches at most 1e-5 of the pixels, each one near-grazing
  (ray within 2 degrees of the oracle patch's tangent plane at the oracle's
  hit, or at the GPU's hit on the oracle's patch of the GPU's cell) or with a
  competing oracle root in the GPU's cell within 1e-4 * extent; where each
  side ray casts its own textures, also a silhouette that the texel
  tolerance moves (the oracle reproduces the GPU's result with its textures
  shifted by that tolerance);
* gradients: ||dg|| / ||g|| <= 1e-3 and per entry |dg| <= 1e-3 max(|g|, 1e-3 ||g||_inf).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import raycast as oray


def device_leaves(scene):
    from paper_2201_10887_amd import api
    w = scene.work
    index = api.build_level_index(scene.leaves, w.side, w.max_depth)
    L = api.DeviceLeaves(scene.leaves, index, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(L)
    return L


def texel_tolerance(leaves, oracle_tex):
    V = float(np.max(np.abs(leaves["v"])))
    return 1e-5 * np.maximum(np.abs(oracle_tex), V)


def grazing_deg(d, tex_k, cas, i, j, t, origin):
    """Angle (degrees) between a ray and the tangent plane of patch (i, j) at the ray point t."""
    p = np.asarray(origin) + t * np.asarray(d)
    u = (p[0] - cas.x0) / cas.hx - i
    v = (p[1] - cas.y0) / cas.hy - j
    h00, h10 = tex_k[j, i], tex_k[j, i + 1]
    h01, h11 = tex_k[j + 1, i], tex_k[j + 1, i + 1]
    dBdx = ((h10 - h00) * (1 - v) + (h11 - h01) * v) / cas.hx
    dBdy = ((h01 - h00) * (1 - u) + (h11 - h10) * u) / cas.hy
    nrm = np.array([-dBdx, -dBdy, 1.0])
    nrm /= np.linalg.norm(nrm)
    return math.degrees(math.asin(min(1.0, abs(float(np.dot(nrm, d))))))


def compare_hits(depth_gpu, hit_gpu, ref, cam, dom, cascades, tex, allow_rate=1e-5, what="", height_tol=0.0):
    """Apply the hit-depth / hit-cell rules; returns (n_mismatch, n_pixels).

    ``height_tol`` > 0 is for comparisons where the two sides ray cast
    different textures (each its own discretization): a mismatch is then also
    explained when the GPU result equals the oracle's result for the oracle
    textures shifted down or up by ``height_tol`` (a silhouette that the
    texel tolerance can move).
    """
    dg = np.asarray(depth_gpu, np.float64).ravel()
    hg = np.asarray(hit_gpu).ravel()
    do, ho = ref["depth"], ref["hit"]
    ext = dom.extent
    n = len(do)
    assert dg.shape == do.shape
    same_hit = hg == ho
    both = np.isfinite(dg) & np.isfinite(do)
    ok_depth = np.zeros(n, dtype=bool)
    ok_depth[both] = np.abs(dg[both] - do[both]) <= 1e-4 * ext
    bad = np.nonzero(~same_hit | (both & ~ok_depth) | (np.isfinite(dg) != np.isfinite(do)))[0]
    o = np.asarray(cam.pos, np.float64)
    shifted = []
    if height_tol > 0 and len(bad):
        for sgn in (-1.0, 1.0):
            r = oray.cast_rays(o, ref["dirs"][bad], dom, cascades, np.asarray(tex) + sgn * height_tol)
            shifted.append(r)
    unexplained = []
    for q, p in enumerate(bad):
        if any((r["hit"][q] == hg[p]) or (np.isfinite(r["depth"][q]) and np.isfinite(dg[p])
                                          and abs(r["depth"][q] - dg[p]) <= 1e-4 * ext)
               or (not np.isfinite(r["depth"][q]) and not np.isfinite(dg[p])) for r in shifted):
            continue
        d = ref["dirs"][p]
        explained = False
        if hg[p] >= 0:
            k, j, i = (int(v[0]) for v in oray.unpack_hit(hg[p:p + 1]))
            t_alt = oray.cell_root(o, d, cascades[k], tex[k], i, j)
            t_ref = do[p] if np.isfinite(do[p]) else dg[p]
            if t_alt is not None and abs(t_alt - t_ref) <= 1e-4 * ext and abs(dg[p] - t_alt) <= 1e-4 * ext:
                explained = True
        if not explained and ho[p] >= 0:
            k, j, i = (int(v[0]) for v in oray.unpack_hit(ho[p:p + 1]))
            if grazing_deg(d, tex[k], cascades[k], i, j, do[p], o) < 2.0:
                explained = True
        if not explained and hg[p] >= 0 and np.isfinite(dg[p]):
            # near-grazing where the GPU hits: the ray meets the oracle's patch of that cell at under 2 degrees
            k, j, i = (int(v[0]) for v in oray.unpack_hit(hg[p:p + 1]))
            if grazing_deg(d, tex[k], cascades[k], i, j, dg[p], o) < 2.0:
                explained = True
        if not explained:
            unexplained.append(int(p))
    detail = []
    for p in unexplained[:6]:
        detail.append(f"[{p}: gpu t={dg[p]:.6g} hit={int(hg[p])} / oracle t={do[p]:.6g} hit={int(ho[p])}]")
    msg = f"{what}: {len(bad)} mismatching pixels of {n}, unexplained {unexplained[:10]} {' '.join(detail)}"
    assert not unexplained, msg
    if allow_rate is not None:
        assert len(bad) <= allow_rate * n, msg
    return len(bad), n


def grad_close(got, ref, rel=1e-3):
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nrm = np.linalg.norm(ref)
    assert nrm > 0
    err = np.linalg.norm(got - ref) / nrm
    per = np.abs(got - ref) <= rel * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return err, per


def hit_grazing_deg(res, cascades, tex, which=0):
    """Per ray of an oracle cast ``res``: the angle (degrees) between the ray and the tangent plane of
    the patch it hits (hit A for which=0, its blend partner B for which=1; NaN where there is none)."""
    rec, val = res["rec"], res["val"]
    k, i, j = rec[:, 4 * which], rec[:, 4 * which + 1], rec[:, 4 * which + 2]
    u, v = val[:, 4 * which + 1], val[:, 4 * which + 2]
    out = np.full(len(k), np.nan)
    has = k >= 0
    if not has.any():
        return out
    kk, ii, jj, uu, vv = k[has], i[has], j[has], u[has], v[has]
    t = np.asarray(tex, np.float64)
    h00, h10 = t[kk, jj, ii], t[kk, jj, ii + 1]
    h01, h11 = t[kk, jj + 1, ii], t[kk, jj + 1, ii + 1]
    hx = np.array([c.hx for c in cascades])[kk]
    hy = np.array([c.hy for c in cascades])[kk]
    bx = ((h10 - h00) * (1 - vv) + (h11 - h01) * vv) / hx
    by = ((h01 - h00) * (1 - uu) + (h11 - h10) * uu) / hy
    d = res["dirs"][has]
    s = np.abs(-bx * d[:, 0] - by * d[:, 1] + d[:, 2]) / np.sqrt(bx * bx + by * by + 1.0)
    out[has] = np.degrees(np.arcsin(np.minimum(s, 1.0)))
    return out


def well_conditioned(res, cascades, tex, min_deg=2.0):
    """Rays whose hits (A and, in a blend, B) meet their patches at min_deg or more: there dt/dh is
    well conditioned.  The complement is the near-grazing set the hit-cell rule also exempts."""
    a = hit_grazing_deg(res, cascades, tex, 0)
    b = hit_grazing_deg(res, cascades, tex, 1)
    return (a >= min_deg) & ~(b < min_deg)
