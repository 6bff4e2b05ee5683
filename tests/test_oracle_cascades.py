"""Pins of the oracle camera and cascade fitting (closed forms and invariants)."""
import math

import numpy as np
import pytest

from oracle import camera, cascades
from paper_2201_10887_amd import synth


def _cam(pos, yaw_deg, pitch_deg, w=320, h=200, vfov_deg=60.0):
    return synth.Camera(pos=pos, yaw=math.radians(yaw_deg), pitch=math.radians(pitch_deg),
                        vfov=math.radians(vfov_deg), width=w, height=h)


def test_camera_frame_and_fov():
    for yaw, pitch in [(0, -20), (37, -5), (200, -70), (-90, 10)]:
        cam = _cam((0, 0, 0), yaw, pitch, 321, 201)
        f, r, u = camera.basis(cam)
        M = np.stack([f, r, u])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(r, f), u) and u[2] > 0 and abs(r[2]) < 1e-15
        # centre pixel of an odd-sized image looks along forward
        d = camera.ray_directions(cam, [160], [100])[0]
        assert np.allclose(d, f, atol=1e-12)
        # top and bottom image edges (centre column) span the vertical field of view
        top, bot = camera.ray_directions(cam, [160, 160], [-0.5, 200.5])
        assert math.isclose(math.acos(np.clip(top @ bot, -1, 1)), cam.vfov, rel_tol=1e-12)
        assert top @ u > 0 > bot @ u
    cam = _cam((0, 0, 0), 0, 0)
    d = camera.ray_directions(cam, [0], [0])[0]
    assert d[0] < 0 and d[2] > 0 and d[1] > 0          # top-left pixel: left, up, forward


def test_log_splits_three_cascades():
    n, f = 37.5, 9100.0
    s = cascades.split_distances(n, f, 3, 1.0, 1.0, 2.0)
    assert math.isclose(s[0], n * (f / n) ** (1 / 3), rel_tol=1e-14)
    assert math.isclose(s[1], n * (f / n) ** (2 / 3), rel_tol=1e-14)
    u = cascades.split_distances(n, f, 4, 0.0, 1.0, 2.0)
    assert np.allclose(u, [n + (f - n) * k / 4 for k in (1, 2, 3)])
    # n below the floor uses n' in the log term only
    s = cascades.split_distances(-5.0, 100.0, 2, 1.0, 1.0, 4.0)
    assert math.isclose(s[0], 4.0 * (100.0 / 4.0) ** 0.5)


def test_flat_box_trapezoid():
    """Flat heightfield, all four frustum edge rays hit the plane inside the domain."""
    dom = synth.Domain(-5000, -5000, 5000, 5000, 0.0, 0.0)
    for yaw in (0.0, 30.0, 145.0):
        cam = _cam((10.0, -20.0, 300.0), yaw, -60.0, 400, 300)
        f, r, u = camera.basis(cam)
        ty = math.tan(cam.vfov / 2)
        tx = ty * cam.width / cam.height
        corners = []
        for sx in (-1, 1):
            for sy in (-1, 1):
                d = f + sx * tx * r + sy * ty * u
                t = -cam.pos[2] / d[2]
                corners.append(np.array(cam.pos[:2]) + t * d[:2])
        hull = cascades.convex_hull(cascades.frustum_box_vertices(cam, dom)[:, :2])
        expect = cascades.convex_hull(np.array(corners))
        assert len(hull) == 4
        assert np.allclose(hull, expect, atol=1e-6)


def _point_in_frustum(cam, p):
    f, r, u = camera.basis(cam)
    q = p - np.asarray(cam.pos)
    c, a, b = q @ f, q @ r, q @ u
    ty = math.tan(cam.vfov / 2)
    tx = ty * cam.width / cam.height
    return (c >= cam.znear) & (np.abs(a) <= c * tx) & (np.abs(b) <= c * ty)


def _inside_convex(poly, pts, tol):
    m = len(poly)
    ok = np.ones(len(pts), dtype=bool)
    for a in range(m):
        p, q = poly[a], poly[(a + 1) % m]
        cross = (q[0] - p[0]) * (pts[:, 1] - p[1]) - (q[1] - p[1]) * (pts[:, 0] - p[0])
        ok &= cross >= -tol
    return ok


CAMS = [((512.0, 51.2, 180.0), 0.0, -20.0), ((512.0, 512.0, 250.0), 33.0, -45.0),
        ((-100.0, 300.0, 400.0), 80.0, -15.0), ((900.0, 900.0, 150.0), 225.0, -5.0),
        ((512.0, 40.0, 120.0), 10.0, -75.0)]


@pytest.mark.parametrize("pos,yaw,pitch", CAMS)
@pytest.mark.parametrize("K,lam", [(2, 1.0), (3, 0.5), (4, 0.0)])
def test_fit_invariants(pos, yaw, pitch, K, lam):
    dom = synth.Domain(0.0, 0.0, 1024.0, 1024.0, 5.0, 300.0)
    cam = _cam(pos, yaw, pitch, 256, 256)
    N, c_min, omega = 256, 16.0, 0.05
    cs = cascades.fit_cascades(cam, dom, K, N, lam, omega, c_min)
    verts = cascades.frustum_box_vertices(cam, dom)
    hull = cascades.convex_hull(verts[:, :2])
    # random points of the box inside the frustum project into the hull
    rng = np.random.default_rng(7)
    P = rng.uniform([dom.x0, dom.y0, dom.zmin], [dom.x1, dom.y1, dom.zmax], size=(20000, 3))
    inside = _point_in_frustum(cam, P)
    assert _inside_convex(hull, P[inside, :2], 1e-6).all()
    # every enumerated vertex lies in the box and (nearly) in the frustum
    f, r, u = camera.basis(cam)
    q = verts - np.asarray(cam.pos)
    ty = math.tan(cam.vfov / 2)
    tx = ty * cam.width / cam.height
    assert np.all(q @ f >= cam.znear - 1e-6)
    assert np.all(np.abs(q @ r) <= (q @ f) * tx + 1e-6) and np.all(np.abs(q @ u) <= (q @ f) * ty + 1e-6)
    assert np.all((verts[:, 0] >= dom.x0 - 1e-6) & (verts[:, 0] <= dom.x1 + 1e-6))
    d = cs[0].offset(hull)
    assert math.isclose(cs[0].near, d.min(), abs_tol=1e-9) and math.isclose(cs[-1].far, d.max(), abs_tol=1e-9)
    for k, c in enumerate(cs):
        if k > 0:
            assert c.near == cs[k - 1].split
        if k < K - 1:
            assert math.isclose(c.far - c.split, omega * (c.split - c.near), rel_tol=1e-12, abs_tol=1e-12)
        # stable fit: lattice origin, even-multiple extents, corners on texel centres
        for o, h, base in ((c.x0, c.hx, dom.x0), (c.y0, c.hy, dom.y0)):
            q = (o - base) / c_min
            assert abs(q - round(q)) < 1e-9
            e = h * (N - 1) / (2 * c_min)
            assert abs(e - round(e)) < 1e-9 and round(e) >= 1
        if len(c.poly):
            assert c.poly[:, 0].min() >= c.x0 - 1e-9 and c.poly[:, 0].max() <= c.x0 + (N - 1) * c.hx + 1e-9
            assert c.poly[:, 1].min() >= c.y0 - 1e-9 and c.poly[:, 1].max() <= c.y0 + (N - 1) * c.hy + 1e-9
            dk = c.offset(c.poly)
            assert dk.min() >= c.near - 1e-9 and dk.max() <= c.far + 1e-9
    # coverage: every hull point is in at least one cascade polygon
    Q = rng.uniform(hull.min(axis=0), hull.max(axis=0), size=(5000, 2))
    Q = Q[_inside_convex(hull, Q, 0.0)]
    covered = np.zeros(len(Q), dtype=bool)
    for c in cs:
        if len(c.poly) >= 3:
            covered |= _inside_convex(c.poly, Q, 1e-7)
    assert covered.all()


def test_fit_rejects_vertical_view():
    dom = synth.Domain(0.0, 0.0, 100.0, 100.0, 0.0, 10.0)
    with pytest.raises(ValueError):
        cascades.fit_cascades(_cam((50, 50, 50), 0, -90), dom, 2, 64, 1.0, 0.05, 1.0)
    with pytest.raises(ValueError):
        cascades.fit_cascades(_cam((50, 50, 50), 0, -30), dom, 2, 60, 1.0, 0.05, 1.0)


def test_fit_misses_box():
    dom = synth.Domain(0.0, 0.0, 100.0, 100.0, 0.0, 10.0)
    cs = cascades.fit_cascades(_cam((50, -500, 50), 180, -10), dom, 3, 64, 1.0, 0.05, 1.0)
    assert all(len(c.poly) == 0 for c in cs)


@pytest.mark.parametrize("pos,yaw,pitch", CAMS)
@pytest.mark.parametrize("N", [64, 256])
def test_aligned_fit_lattice(pos, yaw, pitch, N):
    """Fixed-lattice fit: same polygons as the stable fit; spacing on the quarter-octave ladder,
    origin a whole number of texels from the domain origin, the box covered, and (brute force over
    the ladder) no smaller spacing would cover it."""
    dom = synth.Domain(0.0, 0.0, 1024.0, 1024.0, 5.0, 300.0)
    cam = _cam(pos, yaw, pitch, 256, 256)
    c_min = 16.0
    st = cascades.fit_cascades(cam, dom, 3, N, 0.5, 0.05, c_min)
    al = cascades.fit_cascades(cam, dom, 3, N, 0.5, 0.05, c_min, aligned=True)
    for a, b in zip(st, al):
        assert (a.near, a.far, a.split) == (b.near, b.far, b.split) and np.array_equal(a.poly, b.poly)
        if not len(b.poly):
            continue
        for o, h, base, lo, hi in ((b.x0, b.hx, dom.x0, b.poly[:, 0].min(), b.poly[:, 0].max()),
                                   (b.y0, b.hy, dom.y0, b.poly[:, 1].min(), b.poly[:, 1].max())):
            e = 4.0 * math.log2(h / c_min)
            assert abs(e - round(e)) < 1e-9
            m = (o - base) / h
            assert abs(m - round(m)) < 1e-9
            assert o <= lo + 1e-9 * h and o + (N - 1) * h >= hi - 1e-9 * h
            # the ladder step below fails with its own origin
            hs = c_min * 2.0 ** ((round(e) - 1) / 4.0)
            os_ = base + math.floor((lo - base) / hs + 1e-9) * hs
            assert os_ + (N - 1) * hs < hi - 1e-9 * hs
            assert h < 2.0 ** 0.25 * (hi - lo) / (N - 2) + 1e-9


@pytest.mark.parametrize("pos,yaw,pitch", CAMS)
@pytest.mark.parametrize("N", [64, 256])
def test_stable_fit_is_minimal(pos, yaw, pitch, N):
    """Stable fit (Section 3: corners on the smallest-cell lattice, extents even multiples of it,
    as much of the texture used as possible): the origin is the largest lattice point at or below
    the polygon's box, and the extent the smallest even multiple of c_min reaching past it.  An
    origin one c_min lower, or an extent 2 c_min wider, fails here."""
    dom = synth.Domain(0.0, 0.0, 1024.0, 1024.0, 5.0, 300.0)
    cam = _cam(pos, yaw, pitch, 256, 256)
    c_min = 16.0
    for c in cascades.fit_cascades(cam, dom, 3, N, 0.5, 0.05, c_min):
        if not len(c.poly):
            continue
        for o, h, base, lo, hi in ((c.x0, c.hx, dom.x0, c.poly[:, 0].min(), c.poly[:, 0].max()),
                                   (c.y0, c.hy, dom.y0, c.poly[:, 1].min(), c.poly[:, 1].max())):
            tol = 1e-9 * c_min
            m = (o - base) / c_min
            assert abs(m - round(m)) < 1e-9
            assert o <= lo + tol and o + c_min > lo + tol          # largest lattice point at or below lo
            ext = h * (N - 1)
            e = ext / (2 * c_min)
            assert abs(e - round(e)) < 1e-9 and round(e) >= 1
            assert o + ext >= hi - tol                              # reaches the box
            assert round(e) == 1 or o + ext - 2 * c_min < hi - tol  # and no even multiple less does
