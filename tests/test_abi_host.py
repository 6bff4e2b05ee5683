"""C-ABI library: loads, exports what include/hfr.h declares, host entry points match the oracle.

No GPU needed: only host functions are called, and device entry points are
called with invalid arguments, which are rejected before anything launches.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import cascades as ocas
from oracle import neighbours as onb
from oracle import quadtree as oqt
from paper_2201_10887_amd import _lib, api, synth
from tests import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = _lib.load()
    header = open(os.path.join(ROOT, "include", "hfr.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(hfr_[a-z_0-9]+)\s*\(", header))
    assert len(declared) >= 19
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(_lib.SIGNATURES) == declared
    assert api.abi_version() == 13


@pytest.mark.parametrize("n,depth,tau,seed", [(16, 4, 2.0, 1), (32, 5, 4.0, 2), (64, 4, 0.5, 3), (32, 0, 1.0, 4)])
def test_quadtree_bitexact(n, depth, tau, seed):
    dem = synth.fbm_dem(n, 6, 0.8, seed, zrange=120.0)
    a = api.build_quadtree(dem, 100.0 * n, depth, tau, x0=-50.0, y0=25.0)
    b = oqt.build_quadtree(dem, 100.0 * n, depth, tau, x0=-50.0, y0=25.0)
    for k in ("x", "y", "c", "v", "level", "i", "j"):
        assert np.array_equal(a[k], b[k]), k


def test_quadtree_c1_bitexact(tiny_scene):
    w = tiny_scene.work
    a = api.build_quadtree(tiny_scene.dem, w.side, w.max_depth, w.tau)
    for k in ("x", "y", "c", "v", "level", "i", "j"):
        assert np.array_equal(a[k], tiny_scene.leaves[k]), k


@pytest.mark.parametrize("seed,depth,p,cutoff,sig", [(1, 5, 0.6, 3.5, None), (2, 6, 0.45, 3.0, 1.5),
                                                     (3, 3, 0.9, 2.0, None)])
def test_neighbours_equal_definition(seed, depth, p, cutoff, sig):
    struct = synth.random_leaf_structure(depth, p, seed)
    rng = np.random.default_rng(seed)
    n = len(struct)
    sigma = rng.uniform(0.8, 1.5, n) if sig is None else np.full(n, sig)
    L = synth.leaves_from_structure(struct, 640.0, rng.uniform(0, 200, n), sigma)
    off, idx = api.build_neighbours(L, 640.0, depth, cutoff, 1e-3)
    ref = onb.influence_lists(L, cutoff, 1e-3)
    assert off[0] == 0 and off[-1] == len(idx)
    for i in range(n):
        assert np.array_equal(idx[off[i]:off[i + 1]], ref[i]), i


def test_neighbours_and_locator_c1(tiny_scene):
    w, L = tiny_scene.work, tiny_scene.leaves
    off, idx = api.build_neighbours(L, w.side, w.max_depth, w.cutoff, 1e-3)
    ref = onb.influence_lists(L, w.cutoff, 1e-3)
    assert all(np.array_equal(idx[off[i]:off[i + 1]], ref[i]) for i in range(len(ref)))


@pytest.mark.parametrize("seed,depth,p", [(1, 5, 0.6), (2, 6, 0.45), (3, 0, 0.5)])
def test_level_index(seed, depth, p):
    """Sorted order and per-level prefix counts, written out from their definition."""
    struct = synth.random_leaf_structure(depth, p, seed)
    n = len(struct)
    L = synth.leaves_from_structure(struct, 640.0, np.zeros(n), np.ones(n))
    rank, order = api.build_level_index(L, 640.0, depth)
    assert len(rank) == (4 ** (depth + 1) - 1) // 3 + depth + 1 and len(order) == n
    key = sorted(range(n), key=lambda a: (struct[a][0], struct[a][2], struct[a][1]))
    assert list(order) == key
    want = []
    for l in range(depth + 1):
        S = 2 ** l
        for q in range(S * S + 1):  # leaves of coarser levels, plus level-l leaves before node q
            want.append(sum(1 for (lv, i, j) in struct if lv < l or (lv == l and j * S + i < q)))
    assert np.array_equal(rank, want)


def test_level_index_row_ranges_find_every_leaf():
    """Every leaf is the one leaf of its own node's unit range, empty nodes have empty ranges."""
    struct = synth.random_leaf_structure(6, 0.5, 9)
    n = len(struct)
    L = synth.leaves_from_structure(struct, 64.0, np.zeros(n), np.ones(n))
    rank, order = api.build_level_index(L, 64.0, 6)
    at = {(l, i, j): a for a, (l, i, j) in enumerate(struct)}
    for l in range(7):
        S, off = 2 ** l, api.rank_offset(l)
        for j in range(S):
            for i in range(S):
                q = off + j * S + i
                if (l, i, j) in at:
                    assert rank[q + 1] - rank[q] == 1 and order[rank[q]] == at[(l, i, j)]
                else:
                    assert rank[q + 1] == rank[q]


def test_level_index_rejects_gaps_and_overlaps():
    struct = synth.random_leaf_structure(3, 0.7, 5)
    L = synth.leaves_from_structure(struct[1:], 64.0, np.zeros(len(struct) - 1), np.ones(len(struct) - 1))
    with pytest.raises(_lib.HfrError, match="HFR_EINVAL"):
        api.build_level_index(L, 64.0, 3)
    L2 = synth.leaves_from_structure(struct + [(0, 0, 0)], 64.0, np.zeros(len(struct) + 1), np.ones(len(struct) + 1))
    with pytest.raises(_lib.HfrError, match="HFR_EINVAL"):
        api.build_level_index(L2, 64.0, 3)


def _compare_cascades(a, b, scale):
    assert a.n == b.n
    for f in ("near", "far", "split", "x0", "y0", "hx", "hy"):
        assert abs(getattr(a, f) - getattr(b, f)) <= 1e-9 * scale, f
    assert np.allclose(a.origin, b.origin) and np.allclose(a.vhat, b.vhat, atol=1e-15)
    pa, pb = np.asarray(a.poly), np.asarray(b.poly)
    assert len(pa) > 0 and len(pb) > 0
    # same polygon up to (near-)collinear or duplicate vertices: every vertex of one lies on the other's boundary
    assert _vertex_to_boundary(pa, pb) <= 1e-7 * scale and _vertex_to_boundary(pb, pa) <= 1e-7 * scale


def _vertex_to_boundary(pa, pb):
    worst = 0.0
    for p in pa:
        best = np.inf
        for k in range(len(pb)):
            a, b = pb[k], pb[(k + 1) % len(pb)]
            ab = b - a
            t = 0.0 if not ab.any() else np.clip((p - a) @ ab / (ab @ ab), 0.0, 1.0)
            best = min(best, float(np.linalg.norm(p - (a + t * ab))))
        worst = max(worst, best)
    return worst


CAMERAS = [((512.0, 51.2, 180.0), 0.0, -20.0), ((512.0, 512.0, 250.0), 33.0, -45.0),
           ((-100.0, 300.0, 400.0), 80.0, -15.0), ((900.0, 900.0, 150.0), 225.0, -5.0),
           ((512.0, 40.0, 120.0), 10.0, -75.0), ((512.0, 512.0, 100.0), 0.0, -30.0)]


@pytest.mark.parametrize("pos,yaw,pitch", CAMERAS)
@pytest.mark.parametrize("K,N,lam", [(2, 256, 1.0), (4, 2048, 0.5), (3, 1024, 1.0)])
def test_fit_cascades_matches_oracle(pos, yaw, pitch, K, N, lam):
    dom = synth.Domain(0.0, 0.0, 1024.0, 1024.0, 5.0, 300.0)
    cam = synth.Camera(pos=pos, yaw=math.radians(yaw), pitch=math.radians(pitch), vfov=math.radians(60.0),
                       width=320, height=180)
    got = [api.CascadeView(c) for c in api.fit_cascades(cam, dom, K, N, lam, 0.05, 16.0)]
    ref = ocas.fit_cascades(cam, dom, K, N, lam, 0.05, 16.0)
    for a, b in zip(got, ref):
        _compare_cascades(a, b, dom.extent)


@pytest.mark.parametrize("pos,yaw,pitch", CAMERAS)
@pytest.mark.parametrize("K,N,lam", [(2, 256, 1.0), (4, 2048, 0.5)])
def test_aligned_fit_matches_oracle(pos, yaw, pitch, K, N, lam):
    dom = synth.Domain(0.0, 0.0, 1024.0, 1024.0, 5.0, 300.0)
    cam = synth.Camera(pos=pos, yaw=math.radians(yaw), pitch=math.radians(pitch), vfov=math.radians(60.0),
                       width=320, height=180)
    got = [api.CascadeView(c) for c in api.fit_cascades(cam, dom, K, N, lam, 0.05, 16.0, aligned=True)]
    ref = ocas.fit_cascades(cam, dom, K, N, lam, 0.05, 16.0, aligned=True)
    for a, b in zip(got, ref):
        _compare_cascades(a, b, dom.extent)
        if len(b.poly):  # the ladder step itself is a decision: equal, not merely close
            assert a.hx == b.hx and a.hy == b.hy


def test_fit_cascades_c2_scene():
    dem = synth.fbm_dem(256, 8, 0.8, 1)
    w = synth.MEDIUM
    dom = synth.Domain(0.0, 0.0, w.side, w.side, float(dem.min()), float(dem.max()))
    cam = synth.camera_of(w, dem * 0 + dem)
    got = [api.CascadeView(c) for c in api.fit_cascades(cam, dom, 4, 2048, 0.5, 0.05, 10.0)]
    ref = ocas.fit_cascades(cam, dom, 4, 2048, 0.5, 0.05, 10.0)
    for a, b in zip(got, ref):
        _compare_cascades(a, b, dom.extent)


def _raise_einval(fn, *args):
    lib = _lib.load()
    rc = getattr(lib, fn)(*args)
    assert rc == -1, (fn, rc)
    assert lib.hfr_last_error().decode() != ""


def test_invalid_arguments_rejected_before_launch():
    lib = _lib.load()
    dummy = ctypes.c_void_p(0x1000)
    cam = api.camera(synth.Camera((0, 0, 10), 0.0, -0.3, 1.0, 64, 64))
    dom = api.domain(synth.Domain(0, 0, 100, 100, 0, 10))
    cs = api.fit_cascades(synth.Camera((50, 5, 20), 0.0, -0.3, 1.0, 64, 64), synth.Domain(0, 0, 100, 100, 0, 10),
                          2, 64, 1.0, 0.05, 1.0)
    # maxmip: N not a power of two, K out of range
    _raise_einval("hfr_build_maxmip", dummy, 2, 48, dummy, None)
    _raise_einval("hfr_build_maxmip", dummy, 0, 64, dummy, None)
    _raise_einval("hfr_build_maxmip", dummy, 9, 64, dummy, None)
    # cascades with different N
    bad = (api.Cascade * 2)(cs[0], cs[1])
    bad[1].n = 128
    _raise_einval("hfr_raycast", ctypes.byref(cam), ctypes.byref(dom), bad, 2, dummy, dummy, dummy, dummy, None,
                  None)
    # image too large, NaN camera
    big = api.camera(synth.Camera((0, 0, 10), 0.0, -0.3, 1.0, 20000, 64))
    _raise_einval("hfr_raycast", ctypes.byref(big), ctypes.byref(dom), cs, 2, dummy, dummy, dummy, dummy, None,
                  None)
    nan = api.camera(synth.Camera((float("nan"), 0, 10), 0.0, -0.3, 1.0, 64, 64))
    _raise_einval("hfr_raycast", ctypes.byref(nan), ctypes.byref(dom), cs, 2, dummy, dummy, dummy, dummy, None,
                  None)
    # empty domain
    empty = api.domain(synth.Domain(0, 0, 0, 100, 0, 10))
    _raise_einval("hfr_raycast", ctypes.byref(cam), ctypes.byref(empty), cs, 2, dummy, dummy, dummy, dummy, None,
                  None)
    # discretize: missing level index, bad cutoff, bad depth
    L = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, None, dummy, 4, 3.5, 0.0, 0.0, 1.0)
    _raise_einval("hfr_discretize", ctypes.byref(L), ctypes.byref(dom), cs, 2, dummy, None, None)
    _raise_einval("hfr_discretize", ctypes.byref(api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy,
                                                             dummy, None, 4, 3.5, 0.0, 0.0, 1.0)),
                  ctypes.byref(dom), cs, 2, dummy, None, None)
    L2 = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 4, -1.0, 0.0, 0.0, 1.0)
    _raise_einval("hfr_discretize", ctypes.byref(L2), ctypes.byref(dom), cs, 2, dummy, None, None)
    _raise_einval("hfr_pack_leaves", ctypes.byref(L2), None)
    L3 = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 16, 3.5, 0.0, 0.0, 1.0)
    _raise_einval("hfr_discretize_backward", ctypes.byref(L3), ctypes.byref(dom), cs, 2, dummy, dummy, dummy,
                  dummy, None)
    _raise_einval("hfr_pack_leaves", ctypes.byref(api.Leaves()), None)
    # reuse: no previous frame, or previous textures overlapping the output
    _raise_einval("hfr_discretize_reuse", ctypes.byref(L), ctypes.byref(dom), cs, 2, None, dummy, dummy, None, None,
                  None)
    L5 = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 4, 3.5, 0.0, 0.0, 1.0)
    _raise_einval("hfr_discretize_reuse", ctypes.byref(L5), ctypes.byref(dom), cs, 2, cs, None, dummy, None, None,
                  None)
    _raise_einval("hfr_discretize_reuse", ctypes.byref(L5), ctypes.byref(dom), cs, 2, cs, ctypes.c_void_p(0x1004),
                  dummy, None, None, None)
    # unknown basis
    L4 = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 4, 3.5, 0.0, 0.0, 1.0, 2)
    _raise_einval("hfr_pack_leaves", ctypes.byref(L4), None)
    _raise_einval("hfr_discretize", ctypes.byref(L4), ctypes.byref(dom), cs, 2, dummy, None, None)
    _raise_einval("hfr_discretize_backward", ctypes.byref(L4), ctypes.byref(dom), cs, 2, dummy, dummy, dummy,
                  dummy, None)
    # fit: vertical view, N not a power of two, K out of range
    vert = api.camera(synth.Camera((50, 50, 50), 0.0, -math.pi / 2, 1.0, 64, 64))
    out = (api.Cascade * 8)()
    _raise_einval("hfr_fit_cascades", ctypes.byref(vert), ctypes.byref(dom), 2, 64, 1.0, 0.05, 1.0, out)
    _raise_einval("hfr_fit_cascades", ctypes.byref(cam), ctypes.byref(dom), 2, 60, 1.0, 0.05, 1.0, out)
    _raise_einval("hfr_fit_cascades", ctypes.byref(cam), ctypes.byref(dom), 9, 64, 1.0, 0.05, 1.0, out)
    # quadtree: not a power of two
    q = ctypes.c_void_p()
    dem = np.zeros(9, np.float32)
    _raise_einval("hfr_build_quadtree", dem.ctypes.data_as(ctypes.c_void_p), 3, 1.0, 0.0, 0.0, 1, 0.1,
                  ctypes.byref(q))
    assert lib.hfr_abi_version() == 13


def test_batch_arguments_rejected_before_any_device_call():
    """Every check of hfr_batch_plan_create runs on the host before the plan touches HIP."""
    lib = _lib.load()
    dummy = 0x1000
    dom = api.domain(synth.Domain(0, 0, 100, 100, 0, 10))
    L = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 4, 3.5, 0.0, 0.0, 100.0)
    fields = (_lib.BatchField * 1)()
    fields[0].leaves, fields[0].dom = L, dom

    def view(**kw):
        v = _lib.BatchView(0, 2, 64, 32, 24, 0.5, 0.05, 1.0, dummy, None, dummy, dummy, dummy, None, None)
        for k, x in kw.items():
            setattr(v, k, x)
        return (_lib.BatchView * 1)(v)

    h = ctypes.c_void_p()
    _raise_einval("hfr_batch_plan_create", fields, 1, view(), 0, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 0, view(), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(field=1), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(N=48), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(K=9), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(width=0), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(tex=None), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(c_min=0.0), 1, ctypes.byref(h))
    _raise_einval("hfr_batch_plan_create", fields, 1, view(split_lambda=1.5), 1, ctypes.byref(h))
    bad = (_lib.BatchField * 1)()
    bad[0].leaves, bad[0].dom = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, None, None, 4,
                                           3.5, 0.0, 0.0, 100.0), dom
    _raise_einval("hfr_batch_plan_create", bad, 1, view(), 1, ctypes.byref(h))
    wend = (_lib.BatchField * 1)()
    wend[0].leaves, wend[0].dom = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 4,
                                             3.5, 0.0, 0.0, 100.0, api.BASIS_WENDLAND), dom
    # a Wendland field is accepted by the batch (on a machine without a GPU the plan then fails to allocate)
    rc = lib.hfr_batch_plan_create(wend, 1, view(), 1, ctypes.byref(h))
    assert rc != -5
    if rc == 0:
        lib.hfr_batch_plan_destroy(h)
    h = ctypes.c_void_p()
    bad_basis = (_lib.BatchField * 1)()
    bad_basis[0].leaves, bad_basis[0].dom = api.Leaves(10, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy,
                                                       dummy, 4, 3.5, 0.0, 0.0, 100.0, 7), dom
    _raise_einval("hfr_batch_plan_create", bad_basis, 1, view(), 1, ctypes.byref(h))
    assert h.value is None
    t = _lib.BatchTuning(4, 4, 12, 4, 0, 8)
    _raise_einval("hfr_batch_set_tuning", None, ctypes.byref(t))
    _raise_einval("hfr_batch_long_rays", None, None)
    _raise_einval("hfr_batch_launch", None, None)
    _raise_einval("hfr_batch_launch_backward", None, None)
    _raise_einval("hfr_batch_cascades", None, 0, (api.Cascade * 1)())


@pytest.mark.parametrize("pitch_deg, vfov_deg, height", [(-10.0, 60.0, 1080), (-3.0, 45.0, 720), (5.0, 70.0, 257),
                                                        (-40.0, 30.0, 64)])
@pytest.mark.parametrize("below", [3.0, 8.0, 24.0])
def test_band_rows_follow_the_ray_elevations(pitch_deg, vfov_deg, height, below):
    """api.band_rows (the split ray cast's band): every row above it has its central ray (the oracle's
    camera model) at most `below` degrees under the horizontal, every row from it on more, to within
    the half-row the pixel centres leave."""
    import dataclasses
    from oracle import camera as ocam
    from paper_2201_10887_amd import synth
    cam = synth.Camera(pos=(0.0, 0.0, 100.0), yaw=0.7, pitch=math.radians(pitch_deg), vfov=math.radians(vfov_deg),
                       width=16, height=height)
    rows = api.band_rows(cam, below)
    assert 0 <= rows <= height
    d = ocam.ray_directions(cam, np.full(height, 7.5), np.arange(height, dtype=np.float64))
    # the central column of a 16-wide image: sample between columns 7 and 8 (the image's centre line)
    elev = np.degrees(np.arcsin(d[:, 2] / np.linalg.norm(d, axis=1)))
    slack = 0.5 * vfov_deg / height * 2.0  # one row's angle, generously
    assert np.all(elev[:rows] >= -below - slack)
    assert np.all(elev[rows:] <= -below + slack)
