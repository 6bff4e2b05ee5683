"""GPU parity at the medium scene's full size (3.97M leaves, 4 x 2048^2 cascades, 1920 x 1080).

The GPU runs every kernel over the whole frame in the benchmark's launch
configuration; the oracle recomputes seeded samples of the outputs one by one
(texels, visibility over every cell, rays, gradients restricted to sampled
pixels).  Both sides consume the oracle's leaves and cascades; the library's
own quadtree and cascade fit are checked against them first.
"""
import numpy as np
import pytest

from oracle import adjoint, cascades as ocas, discretize as odisc, maxmip as omip, quadtree as oqt, raycast as oray
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
def medium(gpu):
    w = synth.MEDIUM
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed)
    leaves = oqt.build_quadtree(dem, w.side, w.max_depth, w.tau)
    leaves["sigma"] = np.full(len(leaves["x"]), w.sigma, np.float32)
    dom = synth.Domain(0.0, 0.0, w.side, w.side, float(leaves["v"].min()), float(leaves["v"].max()))
    cam = synth.camera_of(w, dem)
    cs = ocas.fit_cascades(cam, dom, w.cascades, w.tex_n, w.split_lambda, w.overlap, float(leaves["c"].min()))
    index = api.build_level_index(leaves, w.side, w.max_depth)
    L = api.DeviceLeaves(leaves, index, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(L)
    return dict(w=w, dem=dem, leaves=leaves, dom=dom, cam=cam, cs=cs, L=L, cas=api.cascades_from(cs))


def test_library_quadtree_and_fit_match(medium):
    w = medium["w"]
    got = api.build_quadtree(medium["dem"], w.side, w.max_depth, w.tau)
    for k in ("x", "y", "c", "v", "level", "i", "j"):
        assert np.array_equal(got[k], medium["leaves"][k]), k
    fit = api.fit_cascades(medium["cam"], medium["dom"], w.cascades, w.tex_n, w.split_lambda, w.overlap,
                           float(medium["leaves"]["c"].min()))
    for a, b in zip(fit, medium["cs"]):
        for f_lib, f_ora in (("near_d", "near"), ("far_d", "far"), ("split_d", "split"), ("x0", "x0"),
                             ("y0", "y0"), ("hx", "hx"), ("hy", "hy")):
            assert abs(getattr(a, f_lib) - getattr(b, f_ora)) <= 1e-9 * medium["dom"].extent


def test_packed_records_follow_the_level_order(gpu, medium):
    """hfr_pack_leaves: record p holds leaf order[p] (x, y, v exactly, s within one FP32 rounding),
    the level radii are the largest cutoff sigma c per level."""
    m, L, w = medium, medium["L"], medium["w"]
    order = L.order.cpu().numpy()
    packed = L.packed.cpu().numpy()
    lv = m["leaves"]
    for col, key in ((0, "x"), (1, "y"), (2, "v")):
        assert np.array_equal(packed[:, col], lv[key][order]), key
    s = np.sqrt(np.float64(np.log2(np.e) / 2)) / (lv["sigma"][order].astype(np.float64) * lv["c"][order])
    assert np.all(np.abs(packed[:, 3] - s) <= 2 * np.spacing(s.astype(np.float32))), "scale"
    radius = L.level_radius.cpu().numpy()
    for level in range(w.max_depth + 1):
        at = lv["level"] == level
        want = w.cutoff * float((lv["sigma"][at] * lv["c"][at]).max()) if at.any() else 0.0
        assert abs(radius[level] - want * 1.00001) <= 1e-5 * max(want, 1.0), level


def test_wendland_discretize_sampled(gpu, medium):
    """The Wendland basis at the bench's launch shape: sampled texels of all four cascades."""
    m = medium
    W = m["L"].with_basis("wendland")
    api.pack_leaves(W)
    tex = api.discretize(W, m["dom"], m["cas"]).cpu().numpy()
    field = odisc.RBFField(m["leaves"], m["w"].cutoff, "wendland")
    rng = np.random.default_rng(2025)
    for k, cas in enumerate(m["cs"]):
        vis = odisc.visibility(cas)
        assert np.array_equal(vis, np.isfinite(tex[k]))
        jj, ii = np.nonzero(vis)
        pick = rng.choice(len(jj), 2000, replace=False)
        p = odisc.clamp_to_domain(odisc.texel_centres(cas, ii[pick], jj[pick]), m["dom"])
        ref, _ = field.evaluate(p)
        err = np.abs(tex[k][jj[pick], ii[pick]] - ref)
        assert np.all(err <= G.texel_tolerance(m["leaves"], ref)), (k, err.max())
    del W


def test_texel_reuse_next_frame_sampled(gpu, medium):
    """The next frame of a flight built by copying blocks of this one: sampled texels of all four
    cascades against the oracle, and blocks copied."""
    m = medium
    w = m["w"]
    c_min = float(m["leaves"]["c"].min())
    cams = synth.camera_path(m["cam"], 2, step=2.0, yaw_step_deg=0.05)
    cas0, cas1 = (api.fit_cascades(c, m["dom"], w.cascades, w.tex_n, w.split_lambda, w.overlap, c_min, aligned=True)
                  for c in cams)
    tex0 = api.discretize(m["L"], m["dom"], cas0)
    reused = gpu.zeros(1, dtype=gpu.int32, device="cuda")
    tex = api.discretize_reuse(m["L"], m["dom"], cas1, cas0, tex0, reused=reused).cpu().numpy()
    del tex0
    field = odisc.RBFField(m["leaves"], w.cutoff)
    rng = np.random.default_rng(2026)
    blocks = 0
    for k, c in enumerate(cas1):
        cv = api.CascadeView(c)
        vis = odisc.visibility(cv)
        assert np.array_equal(vis, np.isfinite(tex[k]))
        blocks += int(vis.reshape(vis.shape[0] // 16, 16, -1, 16).any(axis=(1, 3)).sum())
        jj, ii = np.nonzero(vis)
        pick = rng.choice(len(jj), 2000, replace=False)
        ref, _ = field.evaluate(odisc.clamp_to_domain(odisc.texel_centres(cv, ii[pick], jj[pick]), m["dom"]))
        err = np.abs(tex[k][jj[pick], ii[pick]] - ref)
        assert np.all(err <= G.texel_tolerance(m["leaves"], ref)), (k, err.max())
    print(f"copied {int(reused.item())} of {blocks} visible blocks", flush=True)
    assert int(reused.item()) > 0


def test_discretize_full_frame_sampled(gpu, medium):
    m = medium
    K, N = len(m["cas"]), m["cas"][0].n
    mask = gpu.zeros((K, N, (N + 31) // 32), dtype=gpu.int32, device="cuda")
    tex = api.discretize(m["L"], m["dom"], m["cas"], mask=mask).cpu().numpy()
    bits = mask.cpu().numpy().view(np.uint32)
    vis_gpu = ((bits[:, :, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(K, N, -1)[:, :, :N].astype(bool)
    assert np.array_equal(vis_gpu, np.isfinite(tex))
    field = odisc.RBFField(m["leaves"], m["w"].cutoff)
    rng = np.random.default_rng(2024)
    for k, cas in enumerate(m["cs"]):
        vis = odisc.visibility(cas)        # every texel of the cascade
        assert np.array_equal(vis, vis_gpu[k]), f"cascade {k}: {np.argwhere(vis != vis_gpu[k])[:5]}"
        jj, ii = np.nonzero(vis)
        pick = rng.choice(len(jj), 4000, replace=False)
        # plus all texels of a few random 8 x 8 tiles and the last row / column
        extra = []
        for _ in range(4):
            a = pick[rng.integers(len(pick))]
            tj, ti = (jj[a] // 8) * 8, (ii[a] // 8) * 8
            extra += [(y, x) for y in range(tj, min(tj + 8, N)) for x in range(ti, min(ti + 8, N)) if vis[y, x]]
        sj = np.concatenate([jj[pick], [e[0] for e in extra]]).astype(np.int64)
        si = np.concatenate([ii[pick], [e[1] for e in extra]]).astype(np.int64)
        p = odisc.clamp_to_domain(odisc.texel_centres(cas, si, sj), m["dom"])
        ref, _ = field.evaluate(p)
        got = tex[k][sj, si]
        tol = G.texel_tolerance(m["leaves"], ref)
        err = np.abs(got - ref)
        assert np.all(err <= tol), f"cascade {k}: max error {err.max()} at {np.argmax(err - tol)}"


@pytest.fixture(scope="module")
def standin(gpu, medium):
    """Stand-in textures of the full frame: the raster sampled at the texels, -inf where invisible."""
    m = medium
    tex = np.stack([synth.resample_raster(m["dem"], m["w"].side, c.x0, c.y0, c.hx, c.hy, c.n) for c in m["cs"]])
    for k, c in enumerate(m["cs"]):
        tex[k][~odisc.visibility(c)] = -np.inf
    return tex


def test_maxmip_full_size_bitexact(gpu, medium, standin):
    mip = api.build_maxmip(gpu.as_tensor(standin, device="cuda")).cpu().numpy()
    for k in range(len(standin)):
        NN = standin.shape[-1] ** 2  # level 0 is not stored
        assert np.array_equal(mip[k][NN:], omip.flatten(omip.maxmip(standin[k]))[NN:].astype(np.float32))


def test_raycast_full_frame_sampled(gpu, medium, standin):
    m = medium
    tex = gpu.as_tensor(standin, device="cuda")
    mip = api.build_maxmip(tex)
    depth, hit = api.raycast(m["cam"], m["dom"], m["cas"], tex, mip)
    depth, hit = depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel()
    cam = m["cam"]
    rng = np.random.default_rng(7)
    pix = rng.choice(cam.width * cam.height, 200_000, replace=False)
    ref = oray.raycast(cam, m["dom"], m["cs"], standin, cols=pix % cam.width, rows=pix // cam.width, threads=16)
    G.compare_hits(depth[pix], hit[pix], ref, cam, m["dom"], m["cs"], standin, what="medium raycast")
    assert np.isfinite(ref["depth"]).mean() > 0.3


def test_long_ray_queue_matches_single_lane_walk(gpu, medium, standin):
    """The queued walk of long rays, lanes sharing each ray, gives the single-lane walk's results."""
    m = medium
    cam = m["cam"]
    tex = gpu.as_tensor(standin, device="cuda")
    mip = api.build_maxmip(tex)
    d0, h0 = api.raycast(cam, m["dom"], m["cas"], tex, mip, work=None)
    work = api.ray_workspace(cam, "cuda")
    d1, h1 = api.raycast(cam, m["dom"], m["cas"], tex, mip, work=work)
    queued = int(work[0].item())
    assert 1000 < queued < cam.width * cam.height // 20, queued  # long rays exist and were queued
    assert int(work[1].item()) == 0  # no ray reached the walk's iteration cap (status word)
    d0, d1, h0, h1 = (a.cpu().numpy() for a in (d0, d1, h0, h1))
    fin = np.isfinite(d0)
    assert np.array_equal(fin, np.isfinite(d1))
    assert (h0 != h1).mean() <= 1e-5
    assert np.max(np.abs(d0[fin] - d1[fin]) / np.abs(d0[fin])) <= 1e-6
    rng = np.random.default_rng(13)
    gd = gpu.as_tensor((rng.normal(0, 1, d0.shape) * fin).astype(np.float32), device="cuda")
    g0 = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip, gd, work=None).cpu().numpy()
    g1 = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip, gd, work=work).cpu().numpy()
    err, per = G.grad_close(g1, g0)
    assert err <= 1e-5 and per.mean() >= 0.9999, (err, per.mean())


@pytest.mark.parametrize("band", ["none", "3deg", "8deg", "half", "all"])
def test_split_frame_matches_single_lane_walk(gpu, medium, standin, band):
    """The frame split at a row (rows above it with the long-ray queue, then their queued rays beside
    the rest): the single-lane walk's results, forward and adjoint, wherever the split falls."""
    m = medium
    cam = m["cam"]
    rows = {"none": 0, "3deg": api.band_rows(cam, 3.0), "8deg": api.band_rows(cam, 8.0), "half": cam.height // 2,
            "all": cam.height}[band]
    tex = gpu.as_tensor(standin, device="cuda")
    mip = api.build_maxmip(tex)
    d0, h0 = api.raycast(cam, m["dom"], m["cas"], tex, mip, work=None)
    work = api.ray_workspace(cam, "cuda")
    d1, h1 = api.raycast(cam, m["dom"], m["cas"], tex, mip, work=work, band_rows=rows)
    queued = int(work[0].item())
    print(f"split at row {rows} of {cam.height}: {queued} rays queued", flush=True)
    assert int(work[1].item()) == 0
    if band in ("8deg", "half", "all"):
        assert queued > 1000, queued  # the band holds the long rays
    d0, d1, h0, h1 = (a.cpu().numpy() for a in (d0, d1, h0, h1))
    fin = np.isfinite(d0)
    assert np.array_equal(fin, np.isfinite(d1))
    assert (h0 != h1).mean() <= 1e-5
    assert np.max(np.abs(d0[fin] - d1[fin]) / np.abs(d0[fin])) <= 1e-6
    rng = np.random.default_rng(13)
    gd = gpu.as_tensor((rng.normal(0, 1, d0.shape) * fin).astype(np.float32), device="cuda")
    g0 = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip, gd, work=None).cpu().numpy()
    g1 = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip, gd, work=work, band_rows=rows).cpu().numpy()
    err, per = G.grad_close(g1, g0)
    assert err <= 1e-5 and per.mean() >= 0.9999, (err, per.mean())


def test_backward_full_frame_sampled(gpu, medium, standin):
    m = medium
    cam = m["cam"]
    K, N = len(m["cas"]), m["cas"][0].n
    tex = gpu.as_tensor(standin, device="cuda")
    mip = api.build_maxmip(tex)
    rng = np.random.default_rng(9)
    pix = rng.choice(cam.width * cam.height, 50_000, replace=False)
    ref = oray.raycast(cam, m["dom"], m["cs"], standin, cols=pix % cam.width, rows=pix // cam.width, threads=16)
    g_pix = rng.normal(0, 1, len(pix)) * np.isfinite(ref["depth"])
    gd = np.zeros(cam.width * cam.height, np.float32)
    gd[pix] = g_pix
    g_ref = adjoint.texel_gradients(ref, g_pix, K, N)
    g_gpu = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip,
                                 gpu.as_tensor(gd.reshape(cam.height, cam.width), device="cuda")).cpu().numpy()
    err, per = G.grad_close(g_gpu, g_ref)
    assert err <= 1e-3 and per.mean() >= 0.999, (err, per.mean())
    # discretize adjoint on the same sparse texel gradient (the stand-in values enter the sigma term)
    field = odisc.RBFField(m["leaves"], m["w"].cutoff)
    gtex32 = g_ref.astype(np.float32)
    gv_ref, gs_ref = adjoint.leaf_gradients(m["cs"], field, m["dom"], gtex32.astype(np.float64))
    # the oracle's sigma term uses the oracle's texel values; feed the GPU those same values
    tex_vals = np.full((K, N, N), -np.inf, np.float32)
    for k, c in enumerate(m["cs"]):
        jj, ii = np.nonzero(gtex32[k] != 0)
        p = odisc.clamp_to_domain(odisc.texel_centres(c, ii, jj), m["dom"])
        tex_vals[k][jj, ii] = field.evaluate(p)[0]
    gv, gs = api.discretize_backward(m["L"], m["dom"], m["cas"], gpu.as_tensor(tex_vals, device="cuda"),
                                     gpu.as_tensor(gtex32, device="cuda"))
    for got, want in ((gv.cpu().numpy(), gv_ref), (gs.cpu().numpy(), gs_ref)):
        err, per = G.grad_close(got, want)
        assert err <= 1e-3 and per.mean() >= 0.999, (err, per.mean())


def test_nearer_surface_composite_sampled(gpu, medium, standin):
    """Two surfaces at full size: the terrain stand-in and a water stand-in above it on part of the
    frame (the terrain plus a seeded smooth rise, below the domain top).  The GPU casts the terrain,
    then the water's nearer pass; sampled pixels against the oracle's per-surface casts composited by
    the nearer hit."""
    from oracle import composite
    m = medium
    rng = np.random.default_rng(31)
    phase = rng.uniform(0, 2 * np.pi, 4)
    water = np.empty_like(standin)
    for k, c in enumerate(m["cs"]):
        x = c.x0 + np.arange(c.n) * c.hx
        y = c.y0 + np.arange(c.n) * c.hy
        X, Y = np.meshgrid(x / 3000.0, y / 3000.0)
        rise = 6.0 * (np.sin(X + phase[0]) * np.cos(Y + phase[1]) + 0.5 * np.sin(2.3 * X + phase[2] + 1.7 * Y))
        water[k] = np.minimum(standin[k] + rise, m["dom"].zmax - 1.0).astype(np.float32)
        water[k][~np.isfinite(standin[k])] = -np.inf
    water = water.astype(np.float32)
    t0, t1 = gpu.as_tensor(standin, device="cuda"), gpu.as_tensor(water, device="cuda")
    m0, m1 = api.build_maxmip(t0), api.build_maxmip(t1)
    work = api.ray_workspace(m["cam"], "cuda")
    depth, hit = api.raycast(m["cam"], m["dom"], m["cas"], t0, m0, work=work)
    api.raycast_nearer(m["cam"], m["dom"], m["cas"], t1, m1, 1, depth, hit, work=work)
    dg, hg = depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel().astype(np.int64)
    cam = m["cam"]
    pix = rng.choice(cam.width * cam.height, 200_000, replace=False)
    rays = [oray.raycast(cam, m["dom"], m["cs"], t, cols=pix % cam.width, rows=pix // cam.width, threads=16)
            for t in (standin, water)]
    comp = composite.nearest(rays)
    assert (comp["surface"] == 1).mean() > 0.05 and (comp["surface"] == 0).mean() > 0.05
    dg, hg = dg[pix], hg[pix]
    sg = np.where(hg >= 0, hg >> composite.SURFACE_SHIFT, -1)
    ext = m["dom"].extent
    differ = np.nonzero(sg != comp["surface"])[0]
    for p in differ:  # a different choice only where both surfaces are hit at (nearly) one depth
        d0, d1 = rays[0]["depth"][p], rays[1]["depth"][p]
        assert np.isfinite(d0) and np.isfinite(d1) and abs(d0 - d1) <= 1e-4 * ext, (p, d0, d1, sg[p])
    assert len(differ) <= 1e-3 * len(pix)
    tag_mask = (1 << composite.SURFACE_SHIFT) - 1
    bad = 0
    for s, tex in ((0, standin), (1, water)):
        sel = np.nonzero((sg == s) & (comp["surface"] == s))[0]
        ref = {key: rays[s][key][sel] for key in ("depth", "hit", "dirs")}
        # every mismatch explained per surface; the rate over all sampled pixels of the frame
        bad += G.compare_hits(dg[sel], hg[sel] & tag_mask, ref, cam, m["dom"], m["cs"], tex, allow_rate=None,
                              what=f"medium surface {s}")[0]
    assert bad <= 1e-5 * len(pix), bad
