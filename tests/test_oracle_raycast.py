"""Pins of the oracle ray caster: closed forms, brute force over cells, dense marching, blend rule."""
import math

import numpy as np
import pytest

from oracle import camera, raycast
from oracle.cascades import Cascade
from paper_2201_10887_amd import synth


def _cascade(near, far, split, x0, y0, hx, hy, n, origin=(0.0, 0.0), vhat=(0.0, 1.0)):
    poly = np.array([[x0, y0], [x0 + (n - 1) * hx, y0], [x0 + (n - 1) * hx, y0 + (n - 1) * hy],
                     [x0, y0 + (n - 1) * hy]])
    return Cascade(near, far, split, np.array(origin, float), np.array(vhat, float) / np.linalg.norm(vhat),
                   x0, y0, hx, hy, n, poly)


def _cam(pos, yaw, pitch, w=64, h=48):
    return synth.Camera(pos=pos, yaw=math.radians(yaw), pitch=math.radians(pitch), vfov=math.radians(60.0),
                        width=w, height=h)


def _bilinear_sample(tex, cas, x, y):
    """Independent bilinear lookup of a texture at world points (nan outside or on invisible cells)."""
    gx = (x - cas.x0) / cas.hx
    gy = (y - cas.y0) / cas.hy
    N = cas.n
    i = np.clip(np.floor(gx).astype(int), 0, N - 2)
    j = np.clip(np.floor(gy).astype(int), 0, N - 2)
    fx, fy = gx - i, gy - j
    v = (tex[j, i] * (1 - fx) * (1 - fy) + tex[j, i + 1] * fx * (1 - fy) + tex[j + 1, i] * (1 - fx) * fy
         + tex[j + 1, i + 1] * fx * fy)
    out = (gx < 0) | (gy < 0) | (gx > N - 1) | (gy > N - 1)
    return np.where(out, np.nan, v)


@pytest.mark.parametrize("a,b,c", [(0.0, 0.0, 40.0), (0.125, -0.0625, 30.0), (-0.25, 0.1875, 90.0)])
@pytest.mark.parametrize("yaw", [0.0, 20.0, -35.0])
def test_tilted_plane_closed_form(a, b, c, yaw):
    N, h = 64, 4.0                   # texel positions and plane values exact in FP32
    cas = _cascade(-1e9, 1e9, 1e9, 0.0, 0.0, h, h, N)
    xs = np.arange(N) * h
    tex = (a * xs[None, :] + b * xs[:, None] + c).astype(np.float32)[None]
    dom = synth.Domain(0.0, 0.0, (N - 1) * h, (N - 1) * h, float(tex.min()), float(tex.max()))
    cam = _cam((128.0, 20.0, 150.0), yaw, -35.0)
    r = raycast.raycast(cam, dom, [cas], tex)
    d = r["dirs"]
    o = np.array(cam.pos)
    t = (o[2] - a * o[0] - b * o[1] - c) / (a * d[:, 0] + b * d[:, 1] - d[:, 2])
    p = o[None, :] + t[:, None] * d
    inside = (t > 0) & (p[:, 0] > 0) & (p[:, 0] < dom.x1) & (p[:, 1] > 0) & (p[:, 1] < dom.y1)
    assert inside.sum() > 100
    assert np.array_equal(np.isfinite(r["depth"]), inside)
    assert np.abs(r["depth"][inside] - t[inside]).max() < 1e-9 * dom.extent
    k, j, i = raycast.unpack_hit(r["hit"][inside])
    gi, gj = p[inside, 0] / h, p[inside, 1] / h
    clear = (np.abs(gi - np.round(gi)) > 1e-6) & (np.abs(gj - np.round(gj)) > 1e-6)
    assert np.array_equal(i[clear], np.floor(gi[clear]).astype(int))
    assert np.array_equal(j[clear], np.floor(gj[clear]).astype(int))
    # the same plane in two overlapping cascades blends two equal hits
    c1 = _cascade(-1e9, 150.0, 140.0, 0.0, 0.0, h, h, N, origin=cam.pos[:2], vhat=(math.sin(math.radians(yaw)), math.cos(math.radians(yaw))))
    c2 = _cascade(140.0, 1e9, 1e9, 0.0, 0.0, h, h, N, origin=cam.pos[:2], vhat=c1.vhat)
    r2 = raycast.raycast(cam, dom, [c1, c2], np.concatenate([tex, tex]))
    assert np.abs(r2["depth"][inside] - t[inside]).max() < 1e-9 * dom.extent
    assert (r2["rec"][:, 4] >= 0).sum() > 0


def _first_hit_bruteforce(o, d, cas, tex, ta, tb, samples=400):
    """Every cell: ray piece in the cell, dense sampling of f then bisection; earliest over cells."""
    N = cas.n
    best = (np.inf, None)
    for j in range(N - 1):
        for i in range(N - 1):
            h = tex[j:j + 2, i:i + 2]
            if not np.all(np.isfinite(h)):
                continue
            lo, hi = ta, tb
            for oo, dd, base, step, m in ((o[0], d[0], cas.x0, cas.hx, i), (o[1], d[1], cas.y0, cas.hy, j)):
                a0, a1 = base + m * step, base + (m + 1) * step
                if dd == 0:
                    if not a0 <= oo <= a1:
                        lo, hi = 1, 0
                    continue
                s0, s1 = sorted(((a0 - oo) / dd, (a1 - oo) / dd))
                lo, hi = max(lo, s0), min(hi, s1)
            if not lo < hi or lo >= best[0]:
                continue

            def f(t):
                x, y = o[0] + t * d[0], o[1] + t * d[1]
                u = (x - (cas.x0 + i * cas.hx)) / cas.hx
                v = (y - (cas.y0 + j * cas.hy)) / cas.hy
                z = h[0, 0] * (1 - u) * (1 - v) + h[0, 1] * u * (1 - v) + h[1, 0] * (1 - u) * v + h[1, 1] * u * v
                return (o[2] + t * d[2]) - z

            ts = np.linspace(lo, hi, samples)
            fs = f(ts)
            below = np.nonzero(fs <= 0)[0]
            if len(below) == 0:
                continue
            q = below[0]
            if q == 0:
                tq = lo
            else:
                a_, b_ = ts[q - 1], ts[q]
                for _ in range(80):
                    m_ = 0.5 * (a_ + b_)
                    if f(m_) <= 0:
                        b_ = m_
                    else:
                        a_ = m_
                tq = b_
            if tq < best[0]:
                best = (tq, (i, j))
    return best


def test_every_cell_bruteforce():
    rng = np.random.default_rng(4)
    N, side = 16, 160.0
    h = side / (N - 1)
    for trial in range(3):
        tex = rng.normal(40.0, 12.0, (N, N)).astype(np.float32)
        if trial == 2:
            tex[rng.random((N, N)) < 0.1] = -np.inf
        cas = _cascade(-1e9, 1e9, 1e9, 0.0, 0.0, h, h, N)
        fin = tex[np.isfinite(tex)]
        dom = synth.Domain(0.0, 0.0, side, side, float(fin.min()), float(fin.max()))
        cam = _cam((80.0 + 10 * trial, -30.0, 110.0), 10.0 * trial - 5, -25.0, 24, 18)
        r = raycast.raycast(cam, dom, [cas], tex[None])
        o = np.array(cam.pos)
        for a in range(len(r["depth"])):
            d = r["dirs"][a]
            # segment: box clip (t >= 0, xy box, z <= zmax)
            ta, tb = 0.0, np.inf
            for oo, dd, lo, hi in ((o[0], d[0], 0.0, side), (o[1], d[1], 0.0, side)):
                s0, s1 = sorted(((lo - oo) / dd, (hi - oo) / dd))
                ta, tb = max(ta, s0), min(tb, s1)
            if d[2] < 0:
                ta = max(ta, (dom.zmax - o[2]) / d[2])
            t_bf, cell = _first_hit_bruteforce(o, d, cas, tex, ta, tb) if ta < tb else (np.inf, None)
            if np.isfinite(t_bf):
                assert abs(r["depth"][a] - t_bf) < 1e-7 * dom.extent
                _, jj, ii = raycast.unpack_hit(r["hit"][a:a + 1])
                if (ii[0], jj[0]) != cell:   # only a shared cell edge may differ
                    p = o + t_bf * d
                    assert min(abs(p[0] / h - round(p[0] / h)), abs(p[1] / h - round(p[1] / h))) < 1e-6
            else:
                assert not np.isfinite(r["depth"][a])


def test_dense_marching_random_scene():
    """March in steps of h/64 over an independent bilinear lookup, then bisect."""
    rng = np.random.default_rng(9)
    N, side = 32, 310.0
    h = side / (N - 1)
    tex = (40 + 25 * np.sin(np.arange(N)[None, :] / 3.0) * np.cos(np.arange(N)[:, None] / 4.0)
           + rng.normal(0, 3, (N, N))).astype(np.float32)
    cas = _cascade(-1e9, 1e9, 1e9, 0.0, 0.0, h, h, N)
    dom = synth.Domain(0.0, 0.0, side, side, float(tex.min()), float(tex.max()))
    cam = _cam((150.0, -10.0, 120.0), 5.0, -20.0, 40, 30)
    r = raycast.raycast(cam, dom, [cas], tex[None])
    o = np.array(cam.pos)
    step = h / 64
    for a in range(0, len(r["depth"]), 3):
        d = r["dirs"][a]
        ts = np.arange(0.0, 1200.0, step)
        P = o[None, :] + ts[:, None] * d[None, :]
        z = _bilinear_sample(tex, cas, P[:, 0], P[:, 1])
        ok = np.isfinite(z) & (P[:, 2] <= dom.zmax)
        below = np.nonzero(ok & (P[:, 2] - z <= 0))[0]
        if len(below) == 0:
            assert not np.isfinite(r["depth"][a]) or r["depth"][a] > 1100
            continue
        q = below[0]
        lo_, hi_ = ts[q - 1], ts[q]
        for _ in range(60):
            m = 0.5 * (lo_ + hi_)
            pm = o + m * d
            if pm[2] - _bilinear_sample(tex, cas, np.array([pm[0]]), np.array([pm[1]]))[0] <= 0:
                hi_ = m
            else:
                lo_ = m
        # marching can step over a thin crest: then the oracle hit is earlier
        assert r["depth"][a] <= hi_ + 1e-9 * dom.extent
        if r["depth"][a] < hi_ - 1e-6 * dom.extent:
            pa = o + r["depth"][a] * d
            za = _bilinear_sample(tex, cas, np.array([pa[0]]), np.array([pa[1]]))[0]
            assert abs(pa[2] - za) < 1e-7 * dom.extent   # a genuine root of the surface
        else:
            assert abs(r["depth"][a] - hi_) < 1e-9 * dom.extent


@pytest.mark.parametrize("reverse", [False, True])
def test_blend_rule_constant_cascades(reverse):
    """Two cascades with different constant heights: depth follows the convex blend in the overlap,
    at its ends and at weights strictly between them (closed-form hits and weights per ray)."""
    N, side = 64, 1000.0
    h = side / (N - 1)
    C1, C2 = 50.0, 45.0
    s, far1 = 300.0, 340.0          # cascade 1: [0, 340], split 300; cascade 2: [300, 1e9]
    cam = _cam((500.0, 100.0, 120.0), 0.0, -8.0, 48, 64)
    vhat = (0.0, -1.0) if reverse else (0.0, 1.0)
    origin = (500.0, 700.0) if reverse else (500.0, 100.0)
    c1 = _cascade(0.0, far1, s, 0.0, 0.0, h, h, N, origin=origin, vhat=vhat)
    c2 = _cascade(s, 1e9, 1e9, 0.0, 0.0, h, h, N, origin=origin, vhat=vhat)
    tex = np.stack([np.full((N, N), C1, np.float32), np.full((N, N), C2, np.float32)])
    dom = synth.Domain(0.0, 0.0, side, side, 40.0, 60.0)
    r = raycast.raycast(cam, dom, [c1, c2], tex)
    d = r["dirs"]
    o = np.array(cam.pos)
    dd = d[:, 0] * c1.vhat[0] + d[:, 1] * c1.vhat[1]
    d0 = (o[0] - origin[0]) * c1.vhat[0] + (o[1] - origin[1]) * c1.vhat[1]
    tA1, tB2 = (o[2] - C1) / -d[:, 2], (o[2] - C2) / -d[:, 2]
    dA1, dB2 = d0 + tA1 * dd, d0 + tB2 * dd
    n_blend = n_inner = 0
    for a in range(len(d)):
        if d[a, 2] >= 0:
            assert not np.isfinite(r["depth"][a])
            continue
        p1 = o + tA1[a] * d[a]
        p2 = o + tB2[a] * d[a]
        in1 = 0 <= dA1[a] <= far1 and 0 <= p1[0] <= side and 0 <= p1[1] <= side
        if not reverse:
            if in1:      # A in cascade 1
                if dA1[a] >= s and s <= dB2[a] <= far1 and 0 <= p2[1] <= side:
                    al = (dA1[a] - s) / (far1 - s)
                    want = (1 - al) * tA1[a] + al * tB2[a]
                    n_blend += 1
                    n_inner += 0.05 < al < 0.95
                else:
                    want = tA1[a]
            else:
                want = tB2[a] if (dB2[a] >= s and 0 <= p2[1] <= side) else np.inf
        else:
            # the ray starts at d = d0 (> far1) in cascade 2 and moves to lower offsets
            in2 = dB2[a] >= s and 0 <= p2[0] <= side and 0 <= p2[1] <= side
            if in2:      # A in cascade 2 (farther); overlap with cascade 1 is [s, far1]
                if dB2[a] <= far1:
                    # partner: first point of cascade 1's overlap part below C1; the ray is
                    # below C1 from tA1 on, and that part starts where d = far1
                    t_far1 = (d0 - far1) / -dd[a]
                    tB = max(tA1[a], t_far1)
                    al = (dB2[a] - s) / (far1 - s)
                    want = (1 - al) * tB + al * tB2[a]
                    n_blend += 1
                    n_inner += 0.05 < al < 0.95
                else:
                    want = tB2[a]
            else:
                want = tA1[a] if in1 else np.inf
        if np.isfinite(want):
            assert abs(r["depth"][a] - want) < 1e-9 * dom.extent, (a, r["depth"][a], want)
        else:
            assert not np.isfinite(r["depth"][a])
    assert n_blend > 0 and n_inner > 0, (n_blend, n_inner)


def test_ray_starting_below_surface_hits_at_entry():
    N = 16
    h = 10.0
    cas = _cascade(-1e9, 1e9, 1e9, 0.0, 0.0, h, h, N)
    tex = np.full((1, N, N), 100.0, np.float32)
    dom = synth.Domain(0.0, 0.0, 150.0, 150.0, 100.0, 100.0)
    cam = _cam((75.0, 75.0, 50.0), 0.0, -10.0, 8, 8)
    r = raycast.raycast(cam, dom, [cas], tex)
    assert np.allclose(r["depth"], 0.0) and np.all(r["rec"][:, 3] == 1)
