"""Pins of the oracle's visibility texture and Eq. 1 / Eq. 2."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import cascades, discretize
from paper_2201_10887_amd import synth


def _leaves_random(depth, p_split, seed, side=512.0, sigma=None):
    struct = synth.random_leaf_structure(depth, p_split, seed)
    rng = np.random.default_rng(seed)
    n = len(struct)
    sig = rng.uniform(0.8, 1.6, n) if sigma is None else np.full(n, sigma)
    return synth.leaves_from_structure(struct, side, rng.uniform(-50, 250, n), sig)


@settings(max_examples=12, deadline=None)
@given(seed=st.integers(0, 10_000), depth=st.integers(2, 6), p=st.floats(0.2, 0.8),
       cutoff=st.sampled_from([2.5, 3.0, 3.5]))
def test_range_query_equals_all_leaves(seed, depth, p, cutoff):
    """Eq. 2 through per-size range queries equals the sum over every leaf (FP64)."""
    L = _leaves_random(depth, p, seed)
    pts = np.random.default_rng(seed + 1).uniform(0, 512.0, (400, 2))
    a, sa = discretize.rbf_bruteforce(pts, L, cutoff)
    b, sb = discretize.RBFField(L, cutoff).evaluate(pts)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * 300) and np.allclose(sa, sb, rtol=1e-12, atol=0)


def test_range_query_equals_all_leaves_c1(tiny_scene):
    s = tiny_scene
    pts = np.random.default_rng(3).uniform(0, s.work.side, (3000, 2))
    a, _ = discretize.rbf_bruteforce(pts, s.leaves, s.work.cutoff)
    b, _ = s.field.evaluate(pts)
    assert np.abs(a - b).max() < 1e-10


def test_weight_closed_form():
    # w at r = 0 is 1 - exp(-k^2/2); at r = k sigma c it is exactly 0; monotone in between
    k = 3.5
    r = np.linspace(0, 3.5 * 1.3 * 20.0, 1001)
    w = discretize.weights(np.zeros((1, 2)), r, np.zeros_like(r), np.full_like(r, 20.0), np.full_like(r, 1.3), k)[0]
    assert math.isclose(w[0], 1 - math.exp(-k * k / 2), rel_tol=1e-15)
    assert w[-1] == 0.0 and np.all(np.diff(w) <= 0) and np.all(w[:-1] > 0)
    # paper's form: exp(-(r/c)^2 / (2 sigma^2)) - exp(-3.5^2/2)
    rr, c, sg = 31.0, 20.0, 1.3
    ref = math.exp(-((rr / c) ** 2) / (2 * sg * sg)) - math.exp(-3.5 ** 2 / 2)
    got = discretize.weights(np.array([[0.0, 0.0]]), [rr], [0.0], [c], [sg], 3.5)[0, 0]
    assert math.isclose(got, ref, rel_tol=1e-14)


@pytest.mark.parametrize("sigma,cutoff", [(1.0, 3.5), (1.5, 3.0), (0.9, 2.0)])
def test_plane_reproduced_on_uniform_grid(sigma, cutoff):
    """Symmetric neighbourhoods cancel first moments: a tilted plane is reproduced exactly."""
    level, side = 5, 640.0
    c = side / 2 ** level
    struct = [(level, i, j) for j in range(2 ** level) for i in range(2 ** level)]
    a, b, c0 = 0.375, -0.1875, 12.5   # exactly representable plane values at the leaf centres
    xs = (np.array([s[1] for s in struct]) + 0.5) * c
    ys = (np.array([s[2] for s in struct]) + 0.5) * c
    L = synth.leaves_from_structure(struct, side, a * xs + b * ys + c0, np.full(len(struct), sigma))
    R = cutoff * sigma * c
    # cell centres, cell corners and edge midpoints, away from the domain edge
    g = np.arange(0.0, side + 1e-9, c / 2)
    px, py = np.meshgrid(g, g)
    pts = np.stack([px.ravel(), py.ravel()], axis=1)
    pts = pts[np.all((pts > R + c) & (pts < side - R - c), axis=1)]
    v, _ = discretize.RBFField(L, cutoff).evaluate(pts)
    assert np.abs(v - (a * pts[:, 0] + b * pts[:, 1] + c0)).max() < 1e-9


def test_bounds_and_truncation(tiny_scene):
    s = tiny_scene
    L = {k: np.asarray(s.leaves[k], np.float64) for k in ("x", "y", "c", "v", "sigma")}
    k = s.work.cutoff
    pts = np.random.default_rng(11).uniform(0, s.work.side, (2000, 2))
    v, s0, (pi, lj, w) = s.field.evaluate(pts, return_terms=True)
    # convex combination of the influencing values
    lo = np.full(len(pts), np.inf)
    hi = np.full(len(pts), -np.inf)
    np.minimum.at(lo, pi, L["v"][lj])
    np.maximum.at(hi, pi, L["v"][lj])
    assert np.all(v >= lo - 1e-9) and np.all(v <= hi + 1e-9)
    # within the stated bound of the untruncated Gaussian sum over all leaves
    r = np.hypot(L["x"][None, :] - pts[:, :1], L["y"][None, :] - pts[:, 1:])
    q = r / (L["sigma"] * L["c"])[None, :]
    gauss = np.exp(-0.5 * q * q)
    trunc = np.maximum(gauss - math.exp(-0.5 * k * k), 0.0)
    vg = (gauss @ L["v"]) / gauss.sum(axis=1)
    bound = np.abs(gauss - trunc).sum(axis=1) / gauss.sum(axis=1) * np.abs(L["v"][None, :] - v[:, None]).max(axis=1)
    assert np.all(np.abs(vg - v) <= bound * (1 + 1e-9) + 1e-9)
    assert np.abs(gauss - trunc).max() <= math.exp(-0.5 * k * k) + 1e-15


def _rect_meets_convex(poly, xa, xb, ya, yb):
    """Brute-force closed rectangle / convex polygon intersection with plain loops."""
    def inside_rect(p):
        return xa <= p[0] <= xb and ya <= p[1] <= yb

    def inside_poly(p):
        m = len(poly)
        if m < 3:
            return False
        s = 0
        for a in range(m):
            q0, q1 = poly[a], poly[(a + 1) % m]
            cr = (q1[0] - q0[0]) * (p[1] - q0[1]) - (q1[1] - q0[1]) * (p[0] - q0[0])
            if cr < 0:
                return False
        return True

    def seg_cross(p1, p2, p3, p4):
        def orient(a, b, c):
            v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
            return 0 if v == 0 else (1 if v > 0 else -1)

        def on(a, b, c):
            return min(a[0], b[0]) <= c[0] <= max(a[0], b[0]) and min(a[1], b[1]) <= c[1] <= max(a[1], b[1])
        o1, o2, o3, o4 = orient(p1, p2, p3), orient(p1, p2, p4), orient(p3, p4, p1), orient(p3, p4, p2)
        if o1 != o2 and o3 != o4:
            return True
        return (o1 == 0 and on(p1, p2, p3)) or (o2 == 0 and on(p1, p2, p4)) or \
               (o3 == 0 and on(p3, p4, p1)) or (o4 == 0 and on(p3, p4, p2))

    rc = [(xa, ya), (xb, ya), (xb, yb), (xa, yb)]
    if any(inside_rect(p) for p in poly) or any(inside_poly(p) for p in rc):
        return True
    m = len(poly)
    for a in range(m):
        for b in range(4):
            if seg_cross(poly[a], poly[(a + 1) % m], rc[b], rc[(b + 1) % 4]):
                return True
    return False


def test_mask_against_bruteforce(tiny_scene):
    s = tiny_scene
    rng = np.random.default_rng(5)
    for cas in s.cascades:
        N = cas.n
        act = discretize.cell_active_sat(cas, *np.meshgrid(np.arange(N - 1), np.arange(N - 1))[::1])
        # sample cells, more of them near the polygon boundary
        ii, jj = rng.integers(0, N - 1, 600), rng.integers(0, N - 1, 600)
        edge = np.argwhere(act != np.roll(act, 1, axis=1))
        pick = edge[rng.integers(0, len(edge), 600)]
        ii = np.concatenate([ii, pick[:, 1]])
        jj = np.concatenate([jj, pick[:, 0]])
        got = discretize.cell_active_sat(cas, ii, jj)
        for a in range(len(ii)):
            xa, xb = cas.x0 + ii[a] * cas.hx, cas.x0 + (ii[a] + 1) * cas.hx
            ya, yb = cas.y0 + jj[a] * cas.hy, cas.y0 + (jj[a] + 1) * cas.hy
            assert got[a] == _rect_meets_convex(cas.poly, xa, xb, ya, yb)
        vis = discretize.visibility(cas)
        assert vis[:-1, :-1][act].all()


def test_invisible_texels_are_minus_inf(tiny_scene):
    for cas, t in zip(tiny_scene.cascades, tiny_scene.tex64):
        vis = discretize.visibility(cas)
        assert np.all(np.isneginf(t[~vis])) and np.all(np.isfinite(t[vis]))
