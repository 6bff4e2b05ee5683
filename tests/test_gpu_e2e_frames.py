"""Whole frames end to end: each side runs its own pipeline on the same seeded inputs.

The GPU renders the frame exactly as the benchmark does (the renderer's own
cascade fit, one discretize launch for all cascades, the max-mipmap, the ray
cast with the long-ray queue); the FP64 oracle fits its own cascades,
evaluates Eq. 2 at every visible texel of them (the plain-C form of the
oracle, Section 4) and ray casts its own FP64 textures (Section 5).  Hit
cells must agree on all but 5e-5 of the pixels, each exception near-grazing
or with a competing root, or a silhouette that the texel tolerance moves
(the oracle reproduces the GPU's result with its textures shifted by it);
depths within 1e-4 of the scene extent.

Scenes: the medium terrain at full size (3.97M leaves, 4 x 2048^2 cascades,
1920 x 1080) and the tiny terrain, every pixel of both.
"""
import os

import numpy as np
import pytest

from oracle import cascades as ocas, discretize as odisc, quadtree as oqt, raycast as oray
from paper_2201_10887_amd import synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
# Hit-cell mismatches allowed when each side casts its own textures: every one must be explained
# (near-grazing, a competing root, or a silhouette the texel tolerance moves).  With the same
# textures the ray casts agree on every sampled pixel; with each side's own textures the FP32
# rounding of the GPU's texels moves a few silhouettes (measured 3.2e-5 of the 1080p frame's
# pixels, 0 on the tiny frame).
E2E_RATE = 5e-5


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle_frame(name, width=None, height=None):
    w = synth.WORKLOADS[name]
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed)
    leaves = oqt.build_quadtree(dem, w.side, w.max_depth, w.tau)
    leaves["sigma"] = np.full(len(leaves["x"]), w.sigma, np.float32)
    dom = synth.Domain(0.0, 0.0, w.side, w.side, float(leaves["v"].min()), float(leaves["v"].max()))
    cam = synth.camera_of(w, dem, width, height)
    cs = ocas.fit_cascades(cam, dom, w.cascades, w.tex_n, w.split_lambda, w.overlap, float(leaves["c"].min()))
    tex = np.stack([odisc.discretize_c(c, leaves, dom, w.cutoff, threads=THREADS) for c in cs])
    return dict(w=w, leaves=leaves, dom=dom, cam=cam, cs=cs, tex=tex)


def _gpu_frame(gpu, f):
    """The benchmark's frame: Renderer.forward with its own fit and the long-ray queue."""
    from paper_2201_10887_amd.renderer import Renderer
    w = f["w"]
    R = Renderer(f["leaves"], w.side, w.max_depth, w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    R.long_ray_queue = True
    depth, hit, cas = R.forward(f["cam"])
    gpu.cuda.synchronize()
    return R, depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel(), cas


def _report(what, nbad, n):
    print(f"{what}: {nbad} hit mismatches of {n} pixels ({nbad / n:.2e})", flush=True)


def test_medium_frame_end_to_end(gpu):
    print("e2e: medium frame (3.97M leaves, 4 x 2048^2, 1920x1080)", flush=True)
    f = _oracle_frame("medium")
    R, depth, hit, cas = _gpu_frame(gpu, f)
    # the two fits agree to rounding (checked in the medium parity tests); both sides own theirs
    assert all(abs(c.x0 - o.x0) <= 1e-9 * f["dom"].extent for c, o in zip(cas, f["cs"]))
    cam = f["cam"]
    ref = oray.raycast(cam, f["dom"], f["cs"], f["tex"], threads=THREADS)  # every pixel
    assert np.isfinite(ref["depth"]).mean() > 0.3
    V = float(np.abs(f["leaves"]["v"]).max())
    nbad, n = G.compare_hits(depth, hit, ref, cam, f["dom"], f["cs"], f["tex"], allow_rate=E2E_RATE,
                             what="medium frame end to end", height_tol=1e-5 * V)
    _report("medium frame", nbad, n)


def test_tiny_frame_end_to_end(gpu):
    print("e2e: tiny frame (2k leaves, 2 x 256^2, 256x256)", flush=True)
    f = _oracle_frame("tiny")
    R, depth, hit, cas = _gpu_frame(gpu, f)
    ref = oray.raycast(f["cam"], f["dom"], f["cs"], f["tex"], threads=THREADS)
    V = float(np.abs(f["leaves"]["v"]).max())
    nbad, n = G.compare_hits(depth, hit, ref, f["cam"], f["dom"], f["cs"], f["tex"], allow_rate=E2E_RATE,
                             what="tiny frame end to end", height_tol=1e-5 * V)
    _report("tiny frame", nbad, n)
