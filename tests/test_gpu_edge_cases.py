"""Edge cases of the device start-up, texel reuse and the second basis: the smallest rasters,
a single leaf, and textures smaller than one 16 x 16 block (every block ragged)."""
import numpy as np
import pytest

from oracle import discretize as odisc, quadtree as oqt
from paper_2201_10887_amd import api, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n,max_depth", [(1, 0), (2, 0), (2, 1), (4, 2)])
def test_smallest_rasters(gpu, n, max_depth):
    dem = np.arange(n * n, dtype=np.float32).reshape(n, n) * 3.0 - 1.0
    dev = api.build_quadtree_device(gpu.as_tensor(dem, device="cuda"), 64.0, max_depth, -1.0, x0=5.0, y0=-7.0)
    ref = oqt.build_quadtree(dem, 64.0, max_depth, -1.0, 5.0, -7.0)
    order = np.lexsort((ref["i"], ref["j"], ref["level"]))
    for k in ("x", "y", "c", "v", "level", "i", "j"):
        assert np.array_equal(dev[k].cpu().numpy(), ref[k][order]), k
    assert dev["x"].numel() == 4 ** max_depth  # tau < 0 refines everywhere
    L = api.DeviceLeaves.from_device(dev, 1.0, 64.0, max_depth, 3.5, 5.0, -7.0)
    api.pack_leaves(L)
    off, idx = api.build_neighbours_device(L)
    host = {k: dev[k].cpu().numpy() for k in ("x", "y", "c")}
    host["sigma"] = np.ones(len(host["x"]), np.float32)
    h_off, h_idx = api.build_neighbours(host, 64.0, max_depth, 3.5, 1e-3, 5.0, -7.0)
    assert np.array_equal(off.cpu().numpy(), h_off.astype(np.int64)) and np.array_equal(idx.cpu().numpy(), h_idx)


@pytest.mark.parametrize("basis", ["gaussian", "wendland"])
def test_reuse_and_basis_on_textures_smaller_than_a_block(gpu, tiny_scene, basis):
    s = tiny_scene
    w = s.work
    L = G.device_leaves(s)
    if basis != "gaussian":
        L = L.with_basis(basis)
        api.pack_leaves(L)
    c_min = float(s.leaves["c"].min())
    cams = synth.camera_path(s.cam, 3, step=40.0)
    field = odisc.RBFField(s.leaves, w.cutoff, basis)
    prev_cas = prev_tex = None
    for cam in cams:
        cas = api.fit_cascades(cam, s.dom, 2, 8, w.split_lambda, w.overlap, c_min, aligned=True)
        if prev_cas is None:
            tex = api.discretize(L, s.dom, cas)
        else:
            tex = api.discretize_reuse(L, s.dom, cas, prev_cas, prev_tex)
        t = tex.cpu().numpy()
        for k, c in enumerate(cas):
            cv = api.CascadeView(c)
            vis = odisc.visibility(cv)
            assert np.array_equal(vis, np.isfinite(t[k]))
            jj, ii = np.nonzero(vis)
            if len(jj):
                ref, _ = field.evaluate(odisc.clamp_to_domain(odisc.texel_centres(cv, ii, jj), s.dom))
                assert np.all(np.abs(t[k][jj, ii] - ref) <= G.texel_tolerance(s.leaves, ref))
        prev_cas, prev_tex = cas, tex
