"""The Wendland C2 basis in the discretization: GPU against the oracle (tiny scene).

Textures at every visible texel and both leaf gradients, to the same bar as the Gaussian
basis; the visibility is the basis's business not at all, so it equals the Gaussian run's; and
switching a leaf set back to the Gaussian reproduces the original records bit for bit.
"""
import numpy as np
import pytest

from oracle import adjoint, discretize as odisc, raycast as oray
from paper_2201_10887_amd import api
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def wend(gpu, tiny_scene):
    s = tiny_scene
    L = G.device_leaves(s)
    W = L.with_basis("wendland")
    api.pack_leaves(W)
    field = odisc.RBFField(s.leaves, s.work.cutoff, "wendland")
    ref = np.stack([odisc.discretize(c, s.leaves, s.dom, s.work.cutoff, field) for c in s.cascades])
    return dict(L=L, W=W, field=field, ref=ref, cas=api.cascades_from(s.cascades))


def test_wendland_textures_match_oracle(gpu, tiny_scene, wend):
    s, ref = tiny_scene, wend["ref"]
    cas = wend["cas"]
    K, N = len(cas), cas[0].n
    mask = gpu.zeros((K, N, (N + 31) // 32), dtype=gpu.int32, device="cuda")
    tex = api.discretize(wend["W"], s.dom, cas, mask=mask).cpu().numpy()
    vis = np.isfinite(ref)
    assert np.array_equal(np.isfinite(tex), vis) and np.array_equal(vis, np.isfinite(s.tex64))
    assert not np.isnan(tex).any()
    err = np.abs(tex[vis] - ref[vis])
    tol = G.texel_tolerance(s.leaves, ref[vis])
    assert np.all(err <= tol), f"max err {err.max()} (tol {tol.min()})"
    # a different surface from the Gaussian one
    assert np.abs(ref[vis] - s.tex64[vis]).max() > 100 * tol.max()
    gauss_mask = gpu.zeros_like(mask)
    api.discretize(wend["L"], s.dom, cas, mask=gauss_mask)
    assert gpu.equal(mask, gauss_mask)


def test_wendland_adjoint_matches_oracle(gpu, tiny_scene, wend):
    s = tiny_scene
    cas = wend["cas"]
    ref32 = wend["ref"].astype(np.float32)
    r = oray.raycast(s.cam, s.dom, s.cascades, ref32, threads=8)
    rng = np.random.default_rng(23)
    gd = rng.normal(0, 1, r["depth"].shape) * np.isfinite(r["depth"])
    gtex = adjoint.texel_gradients(r, gd, len(cas), cas[0].n).astype(np.float32)
    assert np.count_nonzero(gtex) > 1000
    gv_ref, gs_ref = adjoint.leaf_gradients(s.cascades, wend["field"], s.dom, gtex.astype(np.float64))
    gv, gs = api.discretize_backward(wend["W"], s.dom, cas, gpu.as_tensor(ref32, device="cuda"),
                                     gpu.as_tensor(gtex, device="cuda"))
    for got, want in ((gv, gv_ref), (gs, gs_ref)):
        err, per = G.grad_close(got.cpu().numpy(), want)
        assert err <= 1e-3, err
        assert per.mean() >= 0.999, per.mean()


def test_back_to_gaussian_is_bit_identical(gpu, tiny_scene, wend):
    G2 = wend["W"].with_basis("gaussian")
    api.pack_leaves(G2)
    assert gpu.equal(G2.packed, wend["L"].packed) and gpu.equal(G2.level_radius, wend["L"].level_radius)
    assert not gpu.equal(wend["W"].packed[:, 3], wend["L"].packed[:, 3])
    assert gpu.equal(wend["W"].level_radius, wend["L"].level_radius)  # same support radius
