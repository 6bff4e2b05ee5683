"""Pins of the oracle's hand-derived gradients: finite differences and closed forms."""
import numpy as np
import pytest

from oracle import adjoint, camera, cascades, discretize, raycast
from paper_2201_10887_amd import synth
from tests import scenes


def _small_scene(width=48, height=48, N=64):
    s = scenes.oracle_scene("tiny", with_tex=False)
    cam = synth.Camera(s.cam.pos, s.cam.yaw, s.cam.pitch, s.cam.vfov, width, height)
    w = s.work
    cs = cascades.fit_cascades(cam, s.dom, w.cascades, N, w.split_lambda, w.overlap, float(s.leaves["c"].min()))
    return s, cam, cs


def _render(leaves, s, cam, cs, basis="gaussian"):
    field = discretize.RBFField(leaves, s.work.cutoff, basis)
    tex = np.stack([discretize.discretize(c, leaves, s.dom, s.work.cutoff, field) for c in cs])
    return raycast.raycast(cam, s.dom, cs, tex), field, tex


def _hit_ids(r):
    return np.concatenate([r["rec"][:, [0, 1, 2, 4, 5, 6]].ravel()])


def test_texel_gradients_fd():
    s, cam, cs = _small_scene()
    r0, _, tex = _render(s.leaves, s, cam, cs)
    rng = np.random.default_rng(2)
    gd = rng.normal(0, 1, r0["depth"].shape) * np.isfinite(r0["depth"])
    g = adjoint.texel_gradients(r0, gd, len(cs), cs[0].n)
    nz = np.argwhere(g != 0)
    assert len(nz) > 50
    checked = 0
    for k, j, i in nz[rng.choice(len(nz), 40, replace=False)]:
        eps = 1e-4
        tp, tm = tex.copy(), tex.copy()
        tp[k, j, i] += eps
        tm[k, j, i] -= eps
        rp, rm = raycast.raycast(cam, s.dom, cs, tp), raycast.raycast(cam, s.dom, cs, tm)
        if not (np.array_equal(_hit_ids(rp), _hit_ids(r0)) and np.array_equal(_hit_ids(rm), _hit_ids(r0))):
            continue
        fin = np.isfinite(r0["depth"])
        fd = ((rp["depth"][fin] - rm["depth"][fin]) @ gd[fin]) / (2 * eps)
        assert abs(fd - g[k, j, i]) <= 1e-5 * max(abs(g[k, j, i]), 1e-3 * np.abs(g).max())
        checked += 1
    assert checked >= 30


@pytest.mark.parametrize("basis", discretize.BASES)
def test_leaf_gradients_fd(basis):
    s, cam, cs = _small_scene()
    L = {k: np.asarray(v).copy() for k, v in s.leaves.items()}
    rng = np.random.default_rng(1003)
    Lt = dict(L, v=(L["v"] + rng.normal(0, 2.0, len(L["v"]))).astype(np.float32))
    target = _render(Lt, s, cam, cs, basis)[0]["depth"]
    r0, field, _ = _render(L, s, cam, cs, basis)
    loss0, gd = adjoint.l2_loss(r0["depth"], target)
    gtex = adjoint.texel_gradients(r0, gd, len(cs), cs[0].n)
    gv, gs = adjoint.leaf_gradients(cs, field, s.dom, gtex)
    gnorm = max(np.abs(gv).max(), 1e-30)
    cand = np.nonzero(gv != 0)[0]
    assert len(cand) > 40
    checked = 0
    for j in rng.choice(cand, 16, replace=False):
        for name, g, eps in (("v", gv, 1e-4), ("sigma", gs, 1e-5 * float(L["sigma"][j]))):
            Lp = {k: v.astype(np.float64) for k, v in L.items()}
            Lm = {k: v.astype(np.float64) for k, v in L.items()}
            Lp[name][j] += eps
            Lm[name][j] -= eps
            rp, rm = _render(Lp, s, cam, cs, basis)[0], _render(Lm, s, cam, cs, basis)[0]
            if not (np.array_equal(_hit_ids(rp), _hit_ids(r0)) and np.array_equal(_hit_ids(rm), _hit_ids(r0))):
                continue
            fd = (adjoint.l2_loss(rp["depth"], target)[0] - adjoint.l2_loss(rm["depth"], target)[0]) / (2 * eps)
            scale = gnorm if name == "v" else max(np.abs(gs).max(), 1e-30)
            assert abs(fd - g[j]) <= 1e-3 * max(abs(g[j]), 1e-3 * scale), (name, j, fd, g[j])
            checked += 1
    assert checked >= 24


def test_flat_field_closed_forms():
    s, cam, cs = _small_scene(40, 40)
    C = 123.25
    L = {k: np.asarray(v).copy() for k, v in s.leaves.items()}
    L["v"] = np.full(len(L["v"]), C, np.float32)
    dom = synth.Domain(s.dom.x0, s.dom.y0, s.dom.x1, s.dom.y1, C, C + 10.0)   # rays enter above the surface
    field = discretize.RBFField(L, s.work.cutoff)
    tex = np.stack([discretize.discretize(c, L, dom, s.work.cutoff, field) for c in cs])
    fin = np.isfinite(tex)
    assert np.abs(tex[fin] - C).max() < 1e-12
    r = raycast.raycast(cam, dom, cs, tex)
    hit = np.nonzero(np.isfinite(r["depth"]))[0]
    o = np.array(cam.pos)
    dz = r["dirs"][:, 2]
    assert np.abs(r["depth"][hit] - (o[2] - C) / -dz[hit]).max() < 1e-9 * dom.extent
    blended = hit[r["rec"][hit, 4] >= 0]
    picks = np.concatenate([np.random.default_rng(0).choice(hit, 20, replace=False), blended[:10]])
    for p in picks:
        gd = np.zeros(len(r["depth"]))
        gd[p] = 1.0
        gtex = adjoint.texel_gradients(r, gd, len(cs), cs[0].n)
        gv, gs = adjoint.leaf_gradients(cs, field, dom, gtex)
        assert abs(gv.sum() - 1.0 / dz[p]) < 1e-9 * abs(1.0 / dz[p])
        assert np.abs(gs).max() <= 1e-9 * np.abs(gv).max()   # v_j - v_s vanishes up to rounding


def test_stored_fd_probes_match_the_oracle_adjoint():
    """The stored central differences of the differentiable workload's loss (tests/golden/
    c4_tiny512_fd.json, written by tests/golden/make_c4_fd.py from the oracle alone: 64 leaf
    heights, 64 leaf widths) against the oracle's analytic gradient stored beside them: every probe
    within the per-entry rule 1e-3 max(|fd|, 1e-3 max|g|) (measured 4.8e-7 for heights, 8.5e-5 for
    widths).  With the GPU adjoints equal to the oracle's on the oracle's inputs, this closes the
    chain from the GPU gradient to the finite differences probe by probe."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_tiny512_fd.json")
    with open(path) as f:
        gold = json.load(f)
    for which in ("v", "sigma"):
        g = gold[which]
        fd, ana = np.array(g["fd"]), np.array(g["oracle_analytic"])
        assert len(fd) == 64
        rel = np.abs(ana - fd) / np.maximum(np.abs(fd), 1e-3 * g["grad_inf_norm"])
        assert rel.max() <= 1e-3, (which, rel.max())
