"""The batched workload at full size, captured as one graph.

8 seeded fBm heightfields of uneven size (9k to 1.64M leaves, depth 8-12)
and 64 views of them (256^2 to 1920 x 1080, 2-4 cascades, N from the 2^28
texel budget), rendered by the batch launches replayed from a graph:
* every view equals, bit for bit, the per-view entry points run on the
  batch's cascades (textures, pyramids, depth and hit images);
* the 1080p views of the 1.64M-leaf and of the 437k-leaf field against the
  FP64 oracle's own pipeline for that view (its cascade fit, Eq. 2 at every
  visible texel, its ray cast): 200k sampled pixels each, hit cells equal on
  all but 5e-5 of them (each exception near-grazing, with a competing
  root, or a silhouette the texel tolerance moves: the rate of the medium
  frame end to end), depths within 1e-4 of the field's extent.
"""
import os

import numpy as np
import pytest

from oracle import cascades as ocas, discretize as odisc, quadtree as oqt, raycast as oray
from paper_2201_10887_amd import api, autotune, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
SEED = 1004


@pytest.fixture(scope="module")
def c5():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_10887_amd.batch import BatchRenderer, Field, ViewSpec
    print("batch C5: building 8 fields and 64 views", flush=True)
    fspecs = synth.batch_fields(8, SEED)
    vspecs = synth.batch_views(64, 8, SEED)
    dems, leaves, fields = [], [], []
    for f, tau in zip(fspecs, synth.BATCH_TAU):
        dem = synth.fbm_dem(f.dem_n, f.octaves, 0.8, f.seed)
        lv = oqt.build_quadtree(dem, f.side, f.depth, tau)
        lv["sigma"] = np.ones(len(lv["x"]), np.float32)
        dems.append(dem)
        leaves.append(lv)
        fields.append(Field(lv, f.side, f.depth, 3.5, with_grads=False))
    cams = synth.batch_cameras(dems, fspecs, vspecs, SEED)
    ns = autotune.texel_budget([(v.width, v.height, v.K) for v in vspecs], 1 << 28)
    specs = [ViewSpec(v.field, v.K, n, v.width, v.height, 0.5, 0.05) for v, n in zip(vspecs, ns)]
    R = BatchRenderer(fields, specs, backward=False)
    R.set_cameras(cams)
    g = R.capture(backward=False)
    g.replay()
    torch.cuda.synchronize()
    return dict(torch=torch, R=R, cams=cams, leaves=leaves, fspecs=fspecs, fields=fields, graph=g)


def test_every_view_equals_the_per_view_entry_points(c5):
    torch, R, cams = c5["torch"], c5["R"], c5["cams"]
    print(f"batch C5: {R.n_views} views, {sum(s.K * s.N * s.N for s in R.specs)} texels", flush=True)
    for v, (spec, b) in enumerate(zip(R.specs, R.bufs)):
        f = R.fields[spec.field]
        cas = R.cascades(v)
        tex = api.discretize(f.L, f.dom, cas)
        mip = api.build_maxmip(tex)
        depth, hit = api.raycast(cams[v], f.dom, cas, tex, mip, work=None)
        NN = spec.N * spec.N
        assert torch.equal(tex, b["tex"]), v
        assert torch.equal(mip[:, NN:], b["mip"][:, NN:]), v  # level 0 is not stored
        assert torch.equal(hit, b["hit"]), v
        assert torch.equal(torch.nan_to_num(depth, nan=-1.0), torch.nan_to_num(b["depth"], nan=-1.0)), v


@pytest.mark.parametrize("view", [29, 20])
def test_1080p_view_against_the_oracle(c5, view):
    R, cams = c5["R"], c5["cams"]
    spec, cam = R.specs[view], cams[view]
    fs = c5["fspecs"][spec.field]
    lv = c5["leaves"][spec.field]
    assert (cam.width, cam.height) == (1920, 1080) and len(lv["x"]) > 4e5
    print(f"batch C5 view {view}: field {spec.field} ({len(lv['x'])} leaves), K {spec.K}, N {spec.N}", flush=True)
    dom = synth.Domain(0.0, 0.0, fs.side, fs.side, float(lv["v"].min()), float(lv["v"].max()))
    cs = ocas.fit_cascades(cam, dom, spec.K, spec.N, spec.split_lambda, spec.overlap, float(lv["c"].min()))
    for a, b in zip(R.cascades(view), cs):
        assert abs(a.x0 - b.x0) <= 1e-9 * dom.extent and abs(a.hx - b.hx) <= 1e-9 * dom.extent
    otex = np.stack([odisc.discretize_c(c, lv, dom, 3.5, threads=THREADS) for c in cs])
    rng = np.random.default_rng(3000 + view)
    pix = rng.choice(cam.width * cam.height, 200_000, replace=False)
    ref = oray.raycast(cam, dom, cs, otex, cols=pix % cam.width, rows=pix // cam.width, threads=THREADS)
    assert np.isfinite(ref["depth"]).mean() > 0.2
    b = R.bufs[view]
    depth = b["depth"].cpu().numpy().ravel()[pix]
    hit = b["hit"].cpu().numpy().ravel()[pix]
    V = float(np.abs(lv["v"]).max())
    nbad, n = G.compare_hits(depth, hit, ref, cam, dom, cs, otex, allow_rate=5e-5, what=f"batch view {view}",
                             height_tol=1e-5 * V)
    print(f"batch C5 view {view}: {nbad} hit mismatches of {n}", flush=True)


def test_long_ray_queue_keeps_every_view(c5):
    """The same batch with the long-ray queue (eager launches): every view's depth and hit images
    bit-identical to the graph replay's single-lane walks."""
    torch, R = c5["torch"], c5["R"]
    ref = [(b["depth"].clone(), b["hit"].clone()) for b in R.bufs]
    R.set_tuning(ray_queue=1)
    R.forward()
    long_rays = api.batch_long_rays(R.plan)
    torch.cuda.synchronize()
    print(f"batch C5 long-ray queue: {int(long_rays.sum())} rays queued over {int((long_rays > 0).sum())} views",
          flush=True)
    assert long_rays.sum() > 0
    for v, (b, (d, h)) in enumerate(zip(R.bufs, ref)):
        assert torch.equal(torch.nan_to_num(b["depth"], nan=-1.0), torch.nan_to_num(d, nan=-1.0)), v
        assert torch.equal(b["hit"], h), v
    R.set_tuning()
