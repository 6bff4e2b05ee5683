"""GPU parity of two heightfields per frame: terrain and water on the same cells, the nearer drawn.

The water is the seeded stand-in for relative water depths on the terrain's
adaptive grid (Section 2).  Both sides use the oracle's cascades (fitted over
both surfaces' height range) and, per stage, the same oracle-made inputs.
"""
import numpy as np
import pytest

from oracle import adjoint, cascades as ocas, composite, discretize as odisc, raycast as oray
from paper_2201_10887_amd import api, synth
from tests import gpu_common as G
from tests.scenes import oracle_scene

pytestmark = pytest.mark.gpu

WATER_SEED = 77
TAG_MASK = (1 << composite.SURFACE_SHIFT) - 1


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def two(gpu):
    base = oracle_scene("tiny", with_tex=False)
    w, terrain = base.work, base.leaves
    water = dict(terrain)
    water["v"] = synth.water_surface(terrain, w.side, WATER_SEED)
    zmin = float(min(terrain["v"].min(), water["v"].min()))
    zmax = float(max(terrain["v"].max(), water["v"].max()))
    dom = synth.Domain(0.0, 0.0, w.side, w.side, zmin, zmax)
    cs = ocas.fit_cascades(base.cam, dom, w.cascades, w.tex_n, w.split_lambda, w.overlap, float(terrain["c"].min()))
    tex64 = []
    for lv in (terrain, water):
        field = odisc.RBFField(lv, w.cutoff)
        tex64.append(np.stack([odisc.discretize(c, lv, dom, w.cutoff, field) for c in cs]))
    rays = [oray.raycast(base.cam, dom, cs, t.astype(np.float32)) for t in tex64]
    return dict(w=w, leaves=[terrain, water], dom=dom, cam=base.cam, cs=cs, cas=api.cascades_from(cs),
                tex64=tex64, tex32=[t.astype(np.float32) for t in tex64], rays=rays,
                comp=composite.nearest(rays))


def test_water_covers_part_of_the_frame(two):
    seen = two["comp"]["surface"]
    frac = (seen == 1).sum() / max((seen >= 0).sum(), 1)
    assert 0.05 < frac < 0.9, frac


def test_water_discretize_on_shared_cells(gpu, two):
    w, (terrain, water) = two["w"], two["leaves"]
    index = api.build_level_index(terrain, w.side, w.max_depth)
    L0 = api.DeviceLeaves(terrain, index, w.side, w.max_depth, w.cutoff)
    L1 = L0.with_values(water["v"])
    api.pack_leaves(L1)
    tex = api.discretize(L1, two["dom"], two["cas"]).cpu().numpy()
    ref = two["tex64"][1]
    vis = np.isfinite(ref)
    assert np.array_equal(np.isfinite(tex), vis)
    err = np.abs(tex[vis] - ref[vis])
    assert np.all(err <= G.texel_tolerance(water, ref[vis])), err.max()


def _draw(gpu, two, work):
    t0, t1 = (gpu.as_tensor(t, device="cuda") for t in two["tex32"])
    m0, m1 = api.build_maxmip(t0), api.build_maxmip(t1)
    depth, hit = api.raycast(two["cam"], two["dom"], two["cas"], t0, m0, work=work)
    api.raycast_nearer(two["cam"], two["dom"], two["cas"], t1, m1, 1, depth, hit, work=work)
    return (t0, t1), (m0, m1), depth, hit


@pytest.mark.parametrize("queue", [False, True])
def test_nearer_surface_matches_oracle_composite(gpu, two, queue):
    _, _, depth, hit = _draw(gpu, two, api.ray_workspace(two["cam"], "cuda") if queue else None)
    dg, hg = depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel().astype(np.int64)
    comp, rays, ext = two["comp"], two["rays"], two["dom"].extent
    sg = np.where(hg >= 0, hg >> composite.SURFACE_SHIFT, -1)
    # where the two sides pick different surfaces, the two surfaces must be hit at (nearly) one depth
    differ = np.nonzero(sg != comp["surface"])[0]
    for p in differ:
        d0, d1 = rays[0]["depth"][p], rays[1]["depth"][p]
        assert np.isfinite(d0) and np.isfinite(d1) and abs(d0 - d1) <= 1e-4 * ext, (p, d0, d1, sg[p])
    assert len(differ) <= 1e-3 * len(dg)
    for s in (0, 1):
        sel = np.nonzero((sg == s) & (comp["surface"] == s))[0]
        assert len(sel) > 100
        ref = {key: rays[s][key][sel] for key in ("depth", "hit", "dirs")}
        G.compare_hits(dg[sel], hg[sel] & TAG_MASK, ref, two["cam"], two["dom"], two["cs"], two["tex32"][s],
                       what=f"surface {s}")


def test_nearer_surface_adjoints_match_oracle(gpu, two):
    (t0, t1), (m0, m1), depth, hit = _draw(gpu, two, None)
    comp, rays, cam = two["comp"], two["rays"], two["cam"]
    K, N = len(two["cs"]), two["cs"][0].n
    rng = np.random.default_rng(21)
    g = rng.normal(0.0, 1.0, len(comp["depth"])) * np.isfinite(comp["depth"])
    gd = gpu.as_tensor(g.reshape(cam.height, cam.width).astype(np.float32), device="cuda")
    for s, (t, m) in enumerate(((t0, m0), (t1, m1))):
        got = api.raycast_backward_surface(cam, two["dom"], two["cas"], t, m, s, hit, gd, work=None).cpu().numpy()
        ref = adjoint.texel_gradients(rays[s], g * (comp["surface"] == s), K, N)
        err, per = G.grad_close(got, ref)
        assert err <= 1e-3 and per.mean() >= 0.999, (s, err, per.mean())


def test_renderer_draws_both_surfaces(gpu, two):
    from paper_2201_10887_amd.renderer import Renderer
    w, (terrain, water) = two["w"], two["leaves"]
    R = Renderer(terrain, w.side, w.max_depth, w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    assert R.add_surface(water["v"]) == 1
    depth, hit, cas = R.forward(two["cam"])
    # the same kernels on the renderer's own textures, composed by hand
    d0, h0 = api.raycast(two["cam"], R.dom, cas, R.tex, R.mip, work=None)
    d1, h1 = api.raycast(two["cam"], R.dom, cas, R.extra[0]["tex"], R.extra[0]["mip"], work=None)
    d0, d1, h0, h1 = (a.cpu().numpy() for a in (d0, d1, h0, h1))
    want_d = np.where(d1 < d0, d1, d0)
    got = depth.cpu().numpy()
    fin = np.isfinite(want_d)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.max(np.abs(got[fin] - want_d[fin])) <= 1e-6 * two["dom"].extent
    assert ((hit.cpu().numpy() >> composite.SURFACE_SHIFT) == 1).mean() > 0.01
    # the adjoint routes each pixel to the surface it shows
    gd = gpu.isfinite(depth).float()
    gtex = gpu.zeros_like(R.tex)
    gv = gpu.zeros(R.L.n, device="cuda")
    gs = gpu.zeros_like(gv)
    R.backward(two["cam"], cas, gd, gtex, gv, gs, hit=hit)
    assert float(gv.abs().sum()) > 0 and float(R.extra[0]["grad_v"].abs().sum()) > 0


def test_nearer_blend_partner_behind_the_drawn_surface(gpu, two):
    """A second surface 1 mm above the first: in the cascade overlaps its first hit lies in front
    of the first surface's depth and its blend partner (in the next cascade) often behind it.  The
    nearer pass must still blend with that partner, as the oracle's cast of the surface on its own
    does (the adjoint, which walks unclipped, then differentiates the same depth)."""
    t0 = two["tex32"][0]
    t1 = np.where(np.isfinite(t0), t0 + np.float32(1e-3), t0).astype(np.float32)
    cam, dom, cs = two["cam"], two["dom"], two["cs"]
    rays = [oray.raycast(cam, dom, cs, t) for t in (t0, t1)]
    tB = rays[1]["val"][:, 4]
    behind = (rays[1]["rec"][:, 4] >= 0) & (rays[1]["depth"] < rays[0]["depth"]) & (tB > rays[0]["depth"])
    assert behind.sum() > 50, behind.sum()  # the case occurs on this frame
    comp = composite.nearest(rays)
    g0, g1 = gpu.as_tensor(t0, device="cuda"), gpu.as_tensor(t1, device="cuda")
    depth, hit = api.raycast(cam, dom, two["cas"], g0, api.build_maxmip(g0), work=None)
    api.raycast_nearer(cam, dom, two["cas"], g1, api.build_maxmip(g1), 1, depth, hit, work=None)
    dg, hg = depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel().astype(np.int64)
    sel = np.nonzero(behind & (comp["surface"] == 1))[0]
    assert np.all((hg[sel] >> composite.SURFACE_SHIFT) == 1)
    ref = {key: rays[1][key][sel] for key in ("depth", "hit", "dirs")}
    G.compare_hits(dg[sel], hg[sel] & TAG_MASK, ref, cam, dom, cs, t1, what="surface 1 blended behind surface 0")
    # the blend moves these depths by up to ~5 cm, below the depth tolerance: check them to FP32 rounding
    same = (hg[sel] & TAG_MASK) == rays[1]["hit"][sel]
    assert same.mean() >= 0.99
    ext = dom.extent
    assert np.abs(dg[sel][same] - rays[1]["depth"][sel][same]).max() <= 1e-6 * ext
    assert np.abs(rays[1]["depth"][sel] - rays[1]["val"][sel, 0]).max() > 20e-6 * ext  # blended, not t_A
