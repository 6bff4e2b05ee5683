"""Differentiable rendering on the GPU: an image loss taken back to leaf heights and Gaussian widths.

Workload: the tiny heightfield seen at 512 x 512 with its camera; the target
is the FP64 oracle's depth image of the field with every height perturbed by
N(0, 2 m) (seed 1003); the loss is the sum of squared depth differences over
pixels where both images hit.  Checked here:
* the autograd function's gradients equal the adjoint entry points called
  directly with the same depth gradient;
* the gradients agree with the FP64 oracle's analytic gradient of the same
  loss, each side differentiating its own forward pass;
* on 64 seeded leaves for heights and 64 for widths, the GPU gradient agrees
  with central finite differences of the FP64 oracle's loss (eps = 1e-4 m
  for heights, 1e-5 sigma for widths; probes whose +/- eps renders change a
  hit cell are redrawn), stored under tests/golden/ by make_c4_fd.py.
"""
import json
import os

import numpy as np
import pytest

from paper_2201_10887_amd import api
from tests import differentiable as D
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

SIZE = D.SIZE
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c4_tiny512_fd.json")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def problem():
    return D.build_problem()


@pytest.fixture(scope="module")
def gpu_grads(gpu, problem):
    from paper_2201_10887_amd.renderer import Renderer, render_depth
    s = problem["s"]
    w = s.work
    R = Renderer(s.leaves, w.side, w.max_depth, w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    v = gpu.tensor(s.leaves["v"], device="cuda", requires_grad=True)
    sigma = gpu.tensor(s.leaves["sigma"], device="cuda", requires_grad=True)
    target = gpu.as_tensor(problem["target"].reshape(SIZE, SIZE).astype(np.float32), device="cuda")
    depth, hit = render_depth(v, sigma, R, s.cam)
    both = gpu.isfinite(depth) & gpu.isfinite(target)
    diff = gpu.where(both, depth - gpu.where(both, target, gpu.zeros_like(target)), gpu.zeros_like(depth))
    loss = (diff * diff).sum()
    loss.backward()
    gpu.cuda.synchronize()
    return {"R": R, "gv": v.grad.detach().cpu().numpy().astype(np.float64),
            "gs": sigma.grad.detach().cpu().numpy().astype(np.float64), "depth": depth.detach(),
            "diff": diff.detach(), "loss": float(loss)}


def test_autograd_equals_adjoint_entry_points(gpu, problem, gpu_grads):
    s = problem["s"]
    R = gpu_grads["R"]
    cas = R.fit(s.cam)
    gd = (2.0 * gpu_grads["diff"]).contiguous()
    gtex = api.raycast_backward(s.cam, R.dom, cas, R.tex, R.mip, gd)
    gv, gs = api.discretize_backward(R.L, R.dom, cas, R.tex, gtex)
    for got, want in ((gpu_grads["gv"], gv), (gpu_grads["gs"], gs)):
        err, per = G.grad_close(got, want.cpu().numpy())
        assert err <= 1e-5 and per.all(), err


def test_loss_gradient_matches_oracle(problem, gpu_grads):
    """Each side differentiates its own forward pass (textures equal within the texel
    tolerance, depths within the depth tolerance), so the loss gradient per pixel differs
    by up to twice the depth difference: the norm-relative bound holds, and every leaf's
    difference is bounded by 1e-3 of the largest gradient (a leaf whose own gradient is
    small can differ by more than 1e-3 of itself)."""
    assert abs(gpu_grads["loss"] - problem["loss0"]) <= 1e-3 * problem["loss0"]
    for got, want in ((gpu_grads["gv"], problem["gv"]), (gpu_grads["gs"], problem["gs"])):
        err, _ = G.grad_close(got, want)
        assert err <= 1e-3, err
        worst = np.abs(got - want).max() / np.abs(want).max()
        assert worst <= 1e-3, worst


@pytest.mark.parametrize("which", ["v", "sigma"])
def test_gradient_matches_finite_differences(gpu_grads, which):
    with open(GOLDEN) as f:
        gold = json.load(f)[which]
    g_gpu = gpu_grads["gv"] if which == "v" else gpu_grads["gs"]
    leaf = np.array(gold["leaf"])
    fd = np.array(gold["fd"])
    scale = gold["grad_inf_norm"]
    rel = np.abs(g_gpu[leaf] - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
    assert len(leaf) == 64
    assert np.median(rel) <= 1e-3, (np.median(rel), rel.max())
    assert np.mean(rel <= 1e-2) >= 0.95, np.sort(rel)[-5:]
