"""GPU parity at the large scene's full size (64.1M leaves, 4 x 4096^2 cascades, 3840 x 2160).

The GPU runs every kernel over the whole frame; the oracle recomputes seeded
samples: the library's quadtree against the oracle's at full size, visibility
over every texel, texel values in sampled windows (the oracle's Eq. 2 over
every leaf that can reach the window, selected by an exact distance test),
the max-mipmap bit-exact, and sampled rays and their texel gradients on
stand-in textures.  The raster comes from the seeded generator run in torch
on the GPU (the same generator, minutes faster than NumPy at 16384^2).
"""
import numpy as np
import pytest

from oracle import adjoint, cascades as ocas, discretize as odisc, maxmip as omip, quadtree as oqt, raycast as oray
from paper_2201_10887_amd import api, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

THREADS = 16


def _say(msg):
    print(f"[large] {msg}", flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def large(gpu):
    w = synth.LARGE
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed, mountains=w.mountains, device="cuda")
    _say("raster done; oracle quadtree")
    leaves = oqt.build_quadtree(dem, w.side, w.max_depth, w.tau)
    _say(f"{len(leaves['x'])} leaves; cascades, level index, visibility")
    leaves["sigma"] = np.full(len(leaves["x"]), w.sigma, np.float32)
    dom = synth.Domain(0.0, 0.0, w.side, w.side, float(leaves["v"].min()), float(leaves["v"].max()))
    cam = synth.camera_of(w, dem)
    cs = ocas.fit_cascades(cam, dom, w.cascades, w.tex_n, w.split_lambda, w.overlap, float(leaves["c"].min()))
    index = api.build_level_index(leaves, w.side, w.max_depth)
    L = api.DeviceLeaves(leaves, index, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(L)
    del index
    vis = [odisc.visibility(c) for c in cs]  # every texel of every cascade
    _say("scene ready")
    return dict(w=w, dem=dem, leaves=leaves, dom=dom, cam=cam, cs=cs, L=L, cas=api.cascades_from(cs), vis=vis)


def test_scene_size(large):
    n = len(large["leaves"]["x"])
    assert 60e6 < n < 68e6, n


def test_library_quadtree_matches_at_full_size(large):
    w = large["w"]
    got = api.build_quadtree(large["dem"], w.side, w.max_depth, w.tau)
    for k in ("x", "y", "c", "v", "level", "i", "j"):
        assert np.array_equal(got[k], large["leaves"][k]), k


def test_device_quadtree_equals_oracle_at_full_size(gpu, large):
    w = large["w"]
    dev = api.build_quadtree_device(gpu.as_tensor(large["dem"], device="cuda"), w.side, w.max_depth, w.tau)
    lv = large["leaves"]
    order = np.lexsort((lv["i"], lv["j"], lv["level"]))
    for k in ("x", "y", "c", "v", "level", "i", "j"):
        assert np.array_equal(dev[k].cpu().numpy(), lv[k][order]), k


def test_device_neighbour_lists_sampled_at_full_size(gpu, large):
    """The paper's per-leaf influence lists built on the device for the 64.1M device-built leaves
    (3.35G entries): the lists of sampled leaves (every level, plus random ones) against the oracle's
    definition evaluated over all leaves, entry for entry."""
    from oracle import neighbours as onb
    w = large["w"]
    q = api.build_quadtree_device(gpu.as_tensor(large["dem"], device="cuda"), w.side, w.max_depth, w.tau)
    L = api.DeviceLeaves.from_device(q, w.sigma, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(L)
    slack = float(np.float32(1e-3))  # the library takes the slack as a float
    off, idx = api.build_neighbours_device(L, slack)
    _say(f"{idx.numel()} list entries")
    lv = {k: q[k].cpu().numpy() for k in ("x", "y", "c", "level")}
    del q
    x, y, c = (lv[k].astype(np.float64) for k in ("x", "y", "c"))
    R = ((w.cutoff * np.float64(np.float32(w.sigma))) * c) * (1.0 + slack)
    rng = np.random.default_rng(77)
    picks = [int(rng.choice(np.nonzero(lv["level"] == l)[0])) for l in np.unique(lv["level"])]
    picks += [int(p) for p in rng.choice(len(x), 8, replace=False)]
    o = off.cpu().numpy()
    for a in picks:
        d2 = onb.square_distance2(x, y, x[a], y[a], 0.5 * c[a])
        ref = np.nonzero(d2 < R * R)[0]
        got = idx[o[a]:o[a + 1]].cpu().numpy()
        assert np.array_equal(got, ref), (a, int(lv["level"][a]), len(got), len(ref))
    del off, idx, L


def _reaching(leaves, cutoff, box):
    """Indices of every leaf whose truncation radius reaches the closed box (exact test, FP64)."""
    x = leaves["x"].astype(np.float64)
    y = leaves["y"].astype(np.float64)
    r = cutoff * leaves["sigma"].astype(np.float64) * leaves["c"].astype(np.float64) * 1.001
    dx = np.maximum(np.maximum(box[0] - x, x - box[2]), 0.0)
    dy = np.maximum(np.maximum(box[1] - y, y - box[3]), 0.0)
    return np.nonzero(dx * dx + dy * dy < r * r)[0]


def test_discretize_full_frame_sampled(gpu, large):
    m = large
    w = m["w"]
    K, N = len(m["cas"]), m["cas"][0].n
    mask = gpu.zeros((K, N, (N + 31) // 32), dtype=gpu.int32, device="cuda")
    tex = api.discretize(m["L"], m["dom"], m["cas"], mask=mask).cpu().numpy()
    bits = mask.cpu().numpy().view(np.uint32)
    vis_gpu = ((bits[:, :, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(K, N, -1)[:, :, :N].astype(bool)
    assert np.array_equal(vis_gpu, np.isfinite(tex))
    assert not np.isnan(tex).any()
    for k in range(K):
        vis = m["vis"][k]
        assert np.array_equal(vis, vis_gpu[k]), f"cascade {k}: {np.argwhere(vis != vis_gpu[k])[:5]}"
    _check_windows(m, m["cs"], m["vis"], tex, np.random.default_rng(2025))


def _check_windows(m, cascades, vis_all, tex, rng, basis="gaussian", count=3):
    """48 x 48 texel windows around random visible texels of every cascade against the oracle's
    Eq. 2 over every leaf that can reach the window."""
    w = m["w"]
    for k, cas in enumerate(cascades):
        vis = vis_all[k]
        jj, ii = np.nonzero(vis)
        for _ in range(count):
            a = rng.integers(len(jj))
            j0, i0 = max(jj[a] - 24, 0), max(ii[a] - 24, 0)
            wj, wi = np.nonzero(vis[j0:j0 + 48, i0:i0 + 48])
            sj, si = (wj + j0).astype(np.int64), (wi + i0).astype(np.int64)
            p = odisc.clamp_to_domain(odisc.texel_centres(cas, si, sj), m["dom"])
            box = (p[:, 0].min(), p[:, 1].min(), p[:, 0].max(), p[:, 1].max())
            sub = _reaching(m["leaves"], w.cutoff, box)
            field = odisc.RBFField({key: m["leaves"][key][sub] for key in ("x", "y", "c", "v", "sigma")}, w.cutoff,
                                   basis)
            ref, _ = field.evaluate(p)
            got = tex[k][sj, si]
            tol = G.texel_tolerance(m["leaves"], ref)
            err = np.abs(got - ref)
            assert np.all(err <= tol), f"cascade {k}: max error {err.max()} at {np.argmax(err - tol)}"


def test_wendland_discretize_windows(gpu, large):
    m = large
    W = m["L"].with_basis("wendland")
    api.pack_leaves(W)
    tex = api.discretize(W, m["dom"], m["cas"]).cpu().numpy()
    del W
    for k in range(len(m["cs"])):
        assert np.array_equal(np.isfinite(tex[k]), m["vis"][k])
    _check_windows(m, m["cs"], m["vis"], tex, np.random.default_rng(2027), basis="wendland")


def test_texel_reuse_next_frame_windows(gpu, large):
    """The second frame of a flight, built by copying the first frame's blocks, against the oracle."""
    m = large
    w = m["w"]
    c_min = float(m["leaves"]["c"].min())
    cams = synth.camera_path(m["cam"], 2, step=2.0, yaw_step_deg=0.05)
    cas0, cas1 = (api.fit_cascades(c, m["dom"], w.cascades, w.tex_n, w.split_lambda, w.overlap, c_min, aligned=True)
                  for c in cams)
    tex0 = api.discretize(m["L"], m["dom"], cas0)
    reused = gpu.zeros(1, dtype=gpu.int32, device="cuda")
    tex = api.discretize_reuse(m["L"], m["dom"], cas1, cas0, tex0, reused=reused).cpu().numpy()
    del tex0
    views = [api.CascadeView(c) for c in cas1]
    vis = [odisc.visibility(v) for v in views]
    for k in range(len(views)):
        assert np.array_equal(np.isfinite(tex[k]), vis[k]), k
    _say(f"{int(reused.item())} blocks copied")
    assert int(reused.item()) > 0
    _check_windows(m, views, vis, tex, np.random.default_rng(2028))


@pytest.fixture(scope="module")
def standin(gpu, large):
    """Stand-in textures of the full frame: the raster sampled at the texels, -inf where invisible."""
    m = large
    tex = np.stack([synth.resample_raster(m["dem"], m["w"].side, c.x0, c.y0, c.hx, c.hy, c.n) for c in m["cs"]])
    for k in range(len(m["cs"])):
        tex[k][~m["vis"][k]] = -np.inf
    return tex


def test_maxmip_full_size_bitexact(gpu, standin):
    mip = api.build_maxmip(gpu.as_tensor(standin, device="cuda")).cpu().numpy()
    for k in range(len(standin)):
        NN = standin.shape[-1] ** 2  # level 0 is not stored
        assert np.array_equal(mip[k][NN:], omip.flatten(omip.maxmip(standin[k]))[NN:].astype(np.float32))


def test_raycast_full_frame_sampled(gpu, large, standin):
    m = large
    tex = gpu.as_tensor(standin, device="cuda")
    mip = api.build_maxmip(tex)
    depth, hit = api.raycast(m["cam"], m["dom"], m["cas"], tex, mip)
    depth, hit = depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel()
    cam = m["cam"]
    rng = np.random.default_rng(8)
    pix = rng.choice(cam.width * cam.height, 100_000, replace=False)
    ref = oray.raycast(cam, m["dom"], m["cs"], standin, cols=pix % cam.width, rows=pix // cam.width,
                       threads=THREADS)
    G.compare_hits(depth[pix], hit[pix], ref, cam, m["dom"], m["cs"], standin, what="large raycast")
    assert np.isfinite(ref["depth"]).mean() > 0.3


def test_raycast_backward_full_frame_sampled(gpu, large, standin):
    m = large
    cam = m["cam"]
    K, N = len(m["cas"]), m["cas"][0].n
    tex = gpu.as_tensor(standin, device="cuda")
    mip = api.build_maxmip(tex)
    rng = np.random.default_rng(10)
    pix = rng.choice(cam.width * cam.height, 30_000, replace=False)
    ref = oray.raycast(cam, m["dom"], m["cs"], standin, cols=pix % cam.width, rows=pix // cam.width,
                       threads=THREADS)
    g_pix = rng.normal(0, 1, len(pix)) * np.isfinite(ref["depth"])
    gd = np.zeros(cam.width * cam.height, np.float32)
    gd[pix] = g_pix
    g_ref = adjoint.texel_gradients(ref, g_pix, K, N)
    g_gpu = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip,
                                 gpu.as_tensor(gd.reshape(cam.height, cam.width), device="cuda")).cpu().numpy()
    err, per = G.grad_close(g_gpu, g_ref)
    assert err <= 1e-3 and per.mean() >= 0.999, (err, per.mean())


@pytest.fixture(scope="module")
def library_tex(gpu, large):
    """The 4K frame's own textures: the library's Eq. 2 over the 64.1M leaves (pinned to the oracle
    within the texel tolerance by test_discretize_full_frame_sampled), as float32 on both sides."""
    m = large
    tex = api.discretize(m["L"], m["dom"], m["cas"])
    return tex, tex.cpu().numpy()


def test_raycast_on_library_textures_sampled(gpu, large, library_tex):
    """The ray cast of the benchmark's 4K frame on its real, smooth Eq. 2 textures (not the raster
    stand-in): the GPU (with the long-ray queue, as the benchmark runs it) and the FP64 oracle walk
    the same float32 textures; 200k sampled pixels under the hit-cell and depth rules."""
    m = large
    cam = m["cam"]
    tex, tex_h = library_tex
    mip = api.build_maxmip(tex)
    depth, hit = api.raycast(cam, m["dom"], m["cas"], tex, mip)
    depth, hit = depth.cpu().numpy().ravel(), hit.cpu().numpy().ravel()
    rng = np.random.default_rng(18)
    pix = rng.choice(cam.width * cam.height, 200_000, replace=False)
    _say("oracle ray cast of 200k pixels on the library textures")
    ref = oray.raycast(cam, m["dom"], m["cs"], tex_h, cols=pix % cam.width, rows=pix // cam.width, threads=THREADS)
    nbad, n = G.compare_hits(depth[pix], hit[pix], ref, cam, m["dom"], m["cs"], tex_h,
                             what="large raycast on library textures")
    _say(f"{nbad} hit mismatches of {n}")
    assert np.isfinite(ref["depth"]).mean() > 0.3


def test_raycast_backward_on_library_textures_sampled(gpu, large, library_tex):
    m = large
    cam = m["cam"]
    K, N = len(m["cas"]), m["cas"][0].n
    tex, tex_h = library_tex
    mip = api.build_maxmip(tex)
    rng = np.random.default_rng(20)
    pix = rng.choice(cam.width * cam.height, 30_000, replace=False)
    ref = oray.raycast(cam, m["dom"], m["cs"], tex_h, cols=pix % cam.width, rows=pix // cam.width,
                       threads=THREADS)
    g_pix = rng.normal(0, 1, len(pix)) * np.isfinite(ref["depth"])
    gd = np.zeros(cam.width * cam.height, np.float32)
    gd[pix] = g_pix
    g_ref = adjoint.texel_gradients(ref, g_pix, K, N)
    g_gpu = api.raycast_backward(cam, m["dom"], m["cas"], tex, mip,
                                 gpu.as_tensor(gd.reshape(cam.height, cam.width), device="cuda")).cpu().numpy()
    err, per = G.grad_close(g_gpu, g_ref)
    _say(f"adjoint on library textures: norm rel {err:.2e}, per-entry rule on {per.mean():.6f}")
    assert err <= 1e-3 and per.mean() >= 0.999, (err, per.mean())
