"""The differentiable workload shared by the oracle pin, the stored finite differences
and the GPU test: the tiny heightfield seen at 512 x 512 with its camera; the target
is the FP64 oracle's depth image of the field with every height perturbed by N(0, 2 m)
(seed 1003); the loss is the sum of squared depth differences over pixels where both
images hit (oracle only: no value here comes from the HIP library).

``fd`` is a central difference of the oracle's loss for one leaf parameter: it
re-discretizes only the texels the leaf reaches and re-casts only the rays that can
meet them (a superset: a ray is kept when its path up to where its result is decided
crosses the changed texels' box at or below the box's highest texel, a bilinear patch
never exceeding its corners); it returns None when a hit cell changes under +/- eps.
"""
import os

import numpy as np

from oracle import adjoint, discretize as odisc, raycast as oray

SIZE = 512
THREADS = min(16, os.cpu_count() or 1)


def build_problem():
    from tests import scenes
    s = scenes.oracle_scene("tiny", SIZE, SIZE)
    w = s.work
    rng = np.random.default_rng(1003)
    lt = {k: np.array(v) for k, v in s.leaves.items()}
    lt["v"] = (lt["v"] + rng.normal(0.0, 2.0, len(lt["v"]))).astype(np.float32)
    ft = odisc.RBFField(lt, w.cutoff)
    tex_t = np.stack([odisc.discretize(c, lt, s.dom, w.cutoff, ft) for c in s.cascades])
    target = oray.raycast(s.cam, s.dom, s.cascades, tex_t, threads=THREADS)["depth"]
    base = oray.raycast(s.cam, s.dom, s.cascades, s.tex64, threads=THREADS)
    loss0, gd = adjoint.l2_loss(base["depth"], target)
    gtex = adjoint.texel_gradients(base, gd, len(s.cascades), w.tex_n)
    gv_ref, gs_ref = adjoint.leaf_gradients(s.cascades, s.field, s.dom, gtex)
    return {"s": s, "target": target, "base": base, "loss0": loss0, "gv": gv_ref, "gs": gs_ref}


def _search_end(problem):
    """Per ray, a t beyond which nothing can change its result: the first hit t_A, or, when
    t_A lies in an overlap (a second cascade is searched there), the end of that overlap;
    infinity for misses."""
    s, base = problem["s"], problem["base"]
    o = np.asarray(s.cam.pos, np.float64)
    dirs = base["dirs"]
    kA, tA = base["rec"][:, 0], base["val"][:, 0]
    t_end = np.full(len(dirs), np.inf)
    K = len(s.cascades)
    for k, c in enumerate(s.cascades):
        sel = np.nonzero(kA == k)[0]
        if len(sel) == 0:
            continue
        vh = np.asarray(c.vhat)
        d0 = (o[:2] - np.asarray(c.origin)) @ vh
        dd = dirs[sel, :2] @ vh
        dA = d0 + tA[sel] * dd
        fwd = dd >= 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            if k + 1 < K:  # forward sweep: overlap [split_k, far_k] shared with cascade k + 1
                end_f = np.where(dA < c.split, tA[sel], np.maximum(tA[sel], (c.far - d0) / dd))
            else:
                end_f = tA[sel]
            if k > 0:  # backward sweep: overlap [split_{k-1}, far_{k-1}] shared with cascade k - 1
                cp = s.cascades[k - 1]
                end_b = np.where(dA > cp.far, tA[sel], np.maximum(tA[sel], (cp.split - d0) / dd))
            else:
                end_b = tA[sel]
        t_end[sel] = np.where(fwd, end_f, end_b)
    return t_end


def _rays_over_box(o, dirs, t_end, box, zmax):
    """Rays whose path over [0, t_end] crosses the xy box = (x0, y0, x1, y1) at a height
    z <= zmax somewhere (a bilinear patch never exceeds its highest corner)."""
    lo = np.zeros(len(dirs))
    hi = t_end.copy()
    for a, (b0, b1) in enumerate(((box[0], box[2]), (box[1], box[3]))):
        d = dirs[:, a]
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (b0 - o[a]) / d
            t1 = (b1 - o[a]) / d
        inside = (o[a] >= b0) & (o[a] <= b1)
        par = d == 0.0
        lo = np.where(par, np.where(inside, lo, np.inf), np.maximum(lo, np.minimum(t0, t1)))
        hi = np.where(par, hi, np.minimum(hi, np.maximum(t0, t1)))
    hi = np.minimum(hi, 1e7)
    zlow = o[2] + np.minimum(lo * dirs[:, 2], hi * dirs[:, 2])
    return (lo <= hi) & (zlow <= zmax + 1e-6)


def _visible_texels(problem):
    if "vis" not in problem:
        s = problem["s"]
        out = []
        for k, c in enumerate(s.cascades):
            jj, ii = np.nonzero(np.isfinite(s.tex64[k]))
            out.append((jj, ii, odisc.clamp_to_domain(odisc.texel_centres(c, ii, jj), s.dom)))
        problem["vis"] = out
        problem["t_end"] = _search_end(problem)
    return problem["vis"], problem["t_end"]


def fd(problem, j, which, eps):
    """Central difference of the oracle loss for leaf j (re-discretizing only the texels the
    leaf reaches, re-casting only the rays that can meet them); None when a hit cell changes."""
    s = problem["s"]
    w = s.work
    base, target = problem["base"], problem["target"]
    o = np.asarray(s.cam.pos, np.float64)
    dirs = base["dirs"]
    vis, t_end = _visible_texels(problem)
    vals = []
    for sgn in (1.0, -1.0):
        L = {k: np.array(v, np.float64) for k, v in s.leaves.items()}
        L[which][j] += sgn * eps
        field = odisc.RBFField(L, w.cutoff)
        tex = s.tex64.copy()
        R = w.cutoff * float(L["sigma"][j]) * float(L["c"][j]) * 1.001
        pick = np.zeros(len(dirs), bool)
        for k, c in enumerate(s.cascades):
            jj, ii, p = vis[k]
            near = np.hypot(p[:, 0] - L["x"][j], p[:, 1] - L["y"][j]) < R
            if not near.any():
                continue
            tex[k][jj[near], ii[near]] = field.evaluate(p[near])[0]
            i0, i1 = max(ii[near].min() - 1, 0), min(ii[near].max() + 1, c.n - 1)
            j0, j1 = max(jj[near].min() - 1, 0), min(jj[near].max() + 1, c.n - 1)
            win = np.concatenate([tex[k][j0:j1 + 1, i0:i1 + 1].ravel(), s.tex64[k][j0:j1 + 1, i0:i1 + 1].ravel()])
            zmax = float(win[np.isfinite(win)].max())
            box = (c.x0 + i0 * c.hx, c.y0 + j0 * c.hy, c.x0 + i1 * c.hx, c.y0 + j1 * c.hy)
            pick |= _rays_over_box(o, dirs, t_end, box, zmax)
        idx = np.nonzero(pick)[0]
        if len(idx) == 0:
            vals.append(0.0)
            continue
        r = oray.raycast(s.cam, s.dom, s.cascades, tex, cols=base["cols"][idx], rows=base["rows"][idx], threads=THREADS)
        if not np.array_equal(r["hit"], base["hit"][idx]):
            return None
        l_new = adjoint.l2_loss(r["depth"], target[idx])[0]
        l_old = adjoint.l2_loss(base["depth"][idx], target[idx])[0]
        vals.append(l_new - l_old)
    return (vals[0] - vals[1]) / (2.0 * eps)
