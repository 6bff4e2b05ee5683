"""The quadtree built on the device equals the host build (which the oracle pins), in level-index order."""
import numpy as np
import pytest

from paper_2201_10887_amd import api, synth

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "c", "v", "level", "i", "j")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _compare(gpu, dem, side, max_depth, tau, x0=0.0, y0=0.0):
    host = api.build_quadtree(dem, side, max_depth, tau, x0, y0)
    dev = api.build_quadtree_device(gpu.as_tensor(dem, device="cuda"), side, max_depth, tau, x0, y0)
    order = np.lexsort((host["i"], host["j"], host["level"]))  # (level, row, column)
    assert dev["x"].numel() == len(host["x"])
    for k in KEYS:
        assert np.array_equal(dev[k].cpu().numpy(), host[k][order]), k
    rank, _ = api.build_level_index(host, side, max_depth, x0, y0)
    assert np.array_equal(dev["rank"].cpu().numpy(), rank)
    assert np.array_equal(dev["order"].cpu().numpy(), np.arange(len(order)))
    return host, dev


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_device_quadtree_equals_host(gpu, name):
    w = synth.WORKLOADS[name]
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed, mountains=w.mountains)
    host, _ = _compare(gpu, dem, w.side, w.max_depth, w.tau)
    assert len(host["x"]) > 1000


@pytest.mark.parametrize("max_depth,tau", [(0, 1.0), (3, 2.0), (8, 0.5), (8, -1.0)])
def test_device_quadtree_depth_limits_and_origin(gpu, max_depth, tau):
    dem = synth.fbm_dem(256, 6, 0.8, 17)
    _compare(gpu, dem, 512.0, max_depth, tau, x0=-100.0, y0=250.0)


def test_device_built_leaves_discretize_like_host_built(gpu, tiny_scene):
    s = tiny_scene
    w = s.work
    dev = api.build_quadtree_device(gpu.as_tensor(s.dem, device="cuda"), w.side, w.max_depth, w.tau)
    Ld = api.DeviceLeaves.from_device(dev, w.sigma, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(Ld)
    host = api.build_quadtree(s.dem, w.side, w.max_depth, w.tau)
    host["sigma"] = np.full(len(host["x"]), w.sigma, np.float32)
    Lh = api.DeviceLeaves(host, api.build_level_index(host, w.side, w.max_depth), w.side, w.max_depth, w.cutoff)
    api.pack_leaves(Lh)
    assert gpu.equal(Ld.packed, Lh.packed) and gpu.equal(Ld.level_radius, Lh.level_radius)
    cas = api.cascades_from(s.cascades)
    a = api.discretize(Ld, s.dom, cas).cpu().numpy()
    b = api.discretize(Lh, s.dom, cas).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_renderer_from_raster_draws_the_host_built_frame(gpu, tiny_scene):
    from paper_2201_10887_amd.renderer import Renderer
    s = tiny_scene
    w = s.work
    args = (w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    Rh = Renderer(dict(s.leaves), w.side, w.max_depth, *args)
    Rd = Renderer.from_raster(gpu.as_tensor(s.dem, device="cuda"), w.side, w.max_depth, w.tau, w.sigma, *args)
    assert Rd.L.n == Rh.L.n and Rd.c_min == Rh.c_min
    assert (Rd.dom.zmin, Rd.dom.zmax) == (Rh.dom.zmin, Rh.dom.zmax)
    dh, hh, _ = Rh.forward(s.cam)
    dd, hd, _ = Rd.forward(s.cam)
    assert gpu.equal(dd, dh)
    # hit ids name cells by (cascade, texel): the same for both
    assert gpu.equal(hd, hh)


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_device_neighbour_lists_equal_host(gpu, name):
    """Device-built lists over device-built leaves equal the host lists of the same leaves (the host
    lists are pinned to brute force by the oracle tests), entry for entry."""
    w = synth.WORKLOADS[name]
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed, mountains=w.mountains)
    q = api.build_quadtree_device(gpu.as_tensor(dem, device="cuda"), w.side, w.max_depth, w.tau)
    L = api.DeviceLeaves.from_device(q, w.sigma, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(L)
    off, idx = api.build_neighbours_device(L, 1e-3)
    host = {k: q[k].cpu().numpy() for k in ("x", "y", "c")}
    host["sigma"] = np.full(len(host["x"]), w.sigma, np.float32)
    h_off, h_idx = api.build_neighbours(host, w.side, w.max_depth, w.cutoff, 1e-3)
    assert np.array_equal(off.cpu().numpy(), h_off.astype(np.int64))
    assert np.array_equal(idx.cpu().numpy(), h_idx)
