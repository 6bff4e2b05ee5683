"""GPU parity on the tiny scene (1 km fBm, ~2k leaves, 2 x 256^2 cascades, 256 x 256 rays).

Every kernel is compared with the FP64 oracle on the same seeded inputs;
each stage is isolated by feeding both sides the same oracle-made input.
"""
import numpy as np
import pytest

from oracle import adjoint, discretize as odisc, maxmip as omip, raycast as oray
from paper_2201_10887_amd import api, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def dev(gpu, tiny_scene):
    L = G.device_leaves(tiny_scene)
    cas = api.cascades_from(tiny_scene.cascades)
    return L, cas


def test_discretize_matches_oracle(gpu, tiny_scene, dev):
    s = tiny_scene
    L, cas = dev
    K, N = len(cas), cas[0].n
    mask = gpu.zeros((K, N, (N + 31) // 32), dtype=gpu.int32, device="cuda")
    tex = api.discretize(L, s.dom, cas, mask=mask).cpu().numpy()
    gpu.cuda.synchronize()
    ref = s.tex64
    vis_g, vis_o = np.isfinite(tex), np.isfinite(ref)
    assert np.array_equal(vis_g, vis_o), f"visibility differs at {np.argwhere(vis_g != vis_o)[:5]}"
    assert not np.isnan(tex).any()
    err = np.abs(tex[vis_o] - ref[vis_o])
    tol = G.texel_tolerance(s.leaves, ref[vis_o])
    assert np.all(err <= tol), f"max err {err.max()} (tol {tol.min()})"
    assert np.all(np.isneginf(tex[~vis_o]))
    # visibility bits, bit i % 32 of word i / 32
    m = mask.cpu().numpy().view(np.uint32)
    bits = (m[:, :, :, None] >> np.arange(32, dtype=np.uint32)) & 1
    bits = bits.reshape(K, N, -1)[:, :, :N].astype(bool)
    assert np.array_equal(bits, vis_o)


def test_maxmip_bitexact(gpu, tiny_scene):
    tex = gpu.as_tensor(tiny_scene.tex32, device="cuda")
    mip = api.build_maxmip(tex).cpu().numpy()
    for k in range(tex.shape[0]):
        ref = omip.flatten(omip.maxmip(tiny_scene.tex32[k]))
        NN = tiny_scene.tex32.shape[-1] ** 2  # level 0 is not stored
        assert np.array_equal(mip[k][NN:], ref[NN:].astype(np.float32))


@pytest.mark.parametrize("N", [2, 4, 32, 64, 128])
def test_maxmip_small_sizes(gpu, N):
    rng = np.random.default_rng(N)
    t = rng.normal(10, 3, (3, N, N)).astype(np.float32)
    t[rng.random(t.shape) < 0.1] = -np.inf
    mip = api.build_maxmip(gpu.as_tensor(t, device="cuda")).cpu().numpy()
    for k in range(3):
        assert np.array_equal(mip[k][N * N:], omip.flatten(omip.maxmip(t[k]))[N * N:].astype(np.float32))


def test_raycast_matches_oracle(gpu, tiny_scene):
    s = tiny_scene
    cas = api.cascades_from(s.cascades)
    tex = gpu.as_tensor(s.tex32, device="cuda")
    mip = api.build_maxmip(tex)
    depth, hit = api.raycast(s.cam, s.dom, cas, tex, mip)
    ref = oray.raycast(s.cam, s.dom, s.cascades, s.tex32, threads=8)
    nbad, n = G.compare_hits(depth.cpu().numpy(), hit.cpu().numpy(), ref, s.cam, s.dom, s.cascades, s.tex32,
                             what="tiny raycast")
    assert np.isfinite(ref["depth"]).mean() > 0.5


def test_full_frame_matches_oracle(gpu, tiny_scene, dev):
    """Each side runs its own cascade fit, discretization and ray cast."""
    s = tiny_scene
    L, _ = dev
    w = s.work
    cas = api.fit_cascades(s.cam, s.dom, w.cascades, w.tex_n, w.split_lambda, w.overlap, float(s.leaves["c"].min()))
    tex = api.discretize(L, s.dom, cas)
    mip = api.build_maxmip(tex)
    depth, hit = api.raycast(s.cam, s.dom, cas, tex, mip)
    ref = oray.raycast(s.cam, s.dom, s.cascades, s.tex64, threads=8)
    V = float(np.abs(s.leaves["v"]).max())
    G.compare_hits(depth.cpu().numpy(), hit.cpu().numpy(), ref, s.cam, s.dom, s.cascades, s.tex64,
                   allow_rate=1e-5, what="tiny full frame", height_tol=1e-5 * V)


def test_raycast_backward_matches_oracle(gpu, tiny_scene):
    s = tiny_scene
    cas = api.cascades_from(s.cascades)
    tex = gpu.as_tensor(s.tex32, device="cuda")
    mip = api.build_maxmip(tex)
    ref = oray.raycast(s.cam, s.dom, s.cascades, s.tex32, threads=8)
    rng = np.random.default_rng(17)
    gd = (rng.normal(0, 1, ref["depth"].shape) * np.isfinite(ref["depth"])).astype(np.float32)
    g_ref = adjoint.texel_gradients(ref, gd.astype(np.float64), len(cas), cas[0].n)
    g_gpu = api.raycast_backward(s.cam, s.dom, cas, tex, mip,
                                 gpu.as_tensor(gd.reshape(s.cam.height, s.cam.width), device="cuda"))
    err, per = G.grad_close(g_gpu.cpu().numpy(), g_ref)
    assert err <= 1e-3, err
    assert per.mean() >= 0.999, per.mean()


def test_discretize_backward_matches_oracle(gpu, tiny_scene, dev):
    s = tiny_scene
    L, cas = dev
    ref = oray.raycast(s.cam, s.dom, s.cascades, s.tex32, threads=8)
    rng = np.random.default_rng(19)
    gd = rng.normal(0, 1, ref["depth"].shape) * np.isfinite(ref["depth"])
    gtex = adjoint.texel_gradients(ref, gd, len(cas), cas[0].n).astype(np.float32)
    gv_ref, gs_ref = adjoint.leaf_gradients(s.cascades, s.field, s.dom, gtex.astype(np.float64))
    tex = api.discretize(L, s.dom, cas)
    # the forward texel value enters the sigma gradient; give both sides the oracle's
    tex64 = gpu.as_tensor(s.tex32, device="cuda")
    gv, gs = api.discretize_backward(L, s.dom, cas, tex64, gpu.as_tensor(gtex, device="cuda"))
    for got, want in ((gv, gv_ref), (gs, gs_ref)):
        err, per = G.grad_close(got.cpu().numpy(), want)
        assert err <= 1e-3, err
        assert per.mean() >= 0.999, per.mean()
    assert tex.shape == tex64.shape
