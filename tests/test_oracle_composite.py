"""Pins of the oracle's nearest-surface composite: closed-form planes, self-composite, a lifted copy."""
import math

import numpy as np
import pytest

from oracle import composite, raycast
from oracle.cascades import Cascade
from paper_2201_10887_amd import synth


def _plane_scene(a, b, c, N=64, h=4.0):
    poly = np.array([[0.0, 0.0], [(N - 1) * h, 0.0], [(N - 1) * h, (N - 1) * h], [0.0, (N - 1) * h]])
    cas = Cascade(-1e9, 1e9, 1e9, np.zeros(2), np.array([0.0, 1.0]), 0.0, 0.0, h, h, N, poly)
    xs = np.arange(N) * h
    tex = (a * xs[None, :] + b * xs[:, None] + c).astype(np.float32)[None]
    return cas, tex


def _closed_form(o, d, a, b, c):
    """Ray parameter where o + t d meets z = a x + b y + c (the plane extends everywhere)."""
    return (o[2] - a * o[0] - b * o[1] - c) / (a * d[:, 0] + b * d[:, 1] - d[:, 2])


@pytest.mark.parametrize("yaw", [0.0, 25.0])
def test_two_planes_give_the_nearer_closed_form_depth(yaw):
    N, h = 64, 4.0
    terrain = (0.25, -0.125, 30.0)  # rises along x
    water = (0.0, 0.0, 52.0)        # flat: above the terrain on one side, below it on the other
    c1, t1 = _plane_scene(*terrain)
    c2, t2 = _plane_scene(*water)
    zmin = float(min(t1.min(), t2.min()))
    zmax = float(max(t1.max(), t2.max()))
    dom = synth.Domain(0.0, 0.0, (N - 1) * h, (N - 1) * h, zmin, zmax)
    cam = synth.Camera(pos=(126.0, 20.0, 150.0), yaw=math.radians(yaw), pitch=math.radians(-35.0),
                       vfov=math.radians(60.0), width=64, height=48)
    r1 = raycast.raycast(cam, dom, [c1], t1)
    r2 = raycast.raycast(cam, dom, [c2], t2)
    comp = composite.nearest([r1, r2])
    o, d = np.array(cam.pos), r1["dirs"]
    ta, tw = _closed_form(o, d, *terrain), _closed_form(o, d, *water)
    p = lambda t: o[None, :] + t[:, None] * d
    inside = lambda t: (t > 0) & (p(t)[:, 0] > 0) & (p(t)[:, 0] < dom.x1) & (p(t)[:, 1] > 0) & (p(t)[:, 1] < dom.y1)
    ta = np.where(inside(ta), ta, np.inf)
    tw = np.where(inside(tw), tw, np.inf)
    want = np.minimum(ta, tw)
    fin = np.isfinite(want)
    assert fin.sum() > 200
    assert np.array_equal(np.isfinite(comp["depth"]), fin)
    assert np.abs(comp["depth"][fin] - want[fin]).max() < 1e-9 * dom.extent
    # the surface seen is the one with the smaller closed-form depth (away from where they cross)
    clear = fin & (np.abs(ta - tw) > 1e-6 * dom.extent)
    want_s = np.where(tw < ta, 1, 0)
    assert np.array_equal(comp["surface"][clear], want_s[clear])
    assert 0 < (comp["surface"][clear] == 1).mean() < 1
    assert np.array_equal(comp["hit"][fin] >> composite.SURFACE_SHIFT, comp["surface"][fin])


def test_self_composite_and_lifted_copy(tiny_scene):
    s = tiny_scene
    r = raycast.raycast(s.cam, s.dom, s.cascades, s.tex32)
    same = composite.nearest([r, r])
    assert np.array_equal(same["depth"], r["depth"])
    fin = np.isfinite(r["depth"])
    assert np.all(same["surface"][fin] == 0) and np.array_equal(same["hit"], r["hit"])
    # the same textures lifted by 5 m: that surface is hit first wherever the original is
    lifted = s.tex32 + np.float32(5.0)
    dom = synth.Domain(s.dom.x0, s.dom.y0, s.dom.x1, s.dom.y1, s.dom.zmin, s.dom.zmax + 5.0)
    r0 = raycast.raycast(s.cam, dom, s.cascades, s.tex32)
    r1 = raycast.raycast(s.cam, dom, s.cascades, lifted)
    comp = composite.nearest([r0, r1])
    both = np.isfinite(r0["depth"])
    assert np.all(comp["surface"][both] == 1)
    assert np.all(comp["depth"][both] < r0["depth"][both])
