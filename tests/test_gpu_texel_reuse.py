"""Frame-to-frame texel reuse (tiny scene): textures built by copying the previous frame's blocks
match the oracle's Eq. 2 on the new frame's cascades; blocks are copied when and only when the
lattice is shared; nothing is copied from a lattice with another spacing."""
import numpy as np
import pytest

from oracle import cascades as ocas, discretize as odisc
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
def L(gpu, tiny_scene):
    return G.device_leaves(tiny_scene)


def _fit(s, cam):
    w = s.work
    return api.fit_cascades(cam, s.dom, w.cascades, w.tex_n, w.split_lambda, w.overlap,
                            float(s.leaves["c"].min()), aligned=True)


def _check_oracle(s, cas, tex):
    field = s.field
    for k, c in enumerate(cas):
        cv = api.CascadeView(c)
        vis = odisc.visibility(cv)
        assert np.array_equal(vis, np.isfinite(tex[k]))
        jj, ii = np.nonzero(vis)
        ref, _ = field.evaluate(odisc.clamp_to_domain(odisc.texel_centres(cv, ii, jj), s.dom))
        err = np.abs(tex[k][jj, ii] - ref)
        assert np.all(err <= G.texel_tolerance(s.leaves, ref)), (k, err.max())


def test_reuse_along_a_flight(gpu, tiny_scene, L):
    s = tiny_scene
    path = synth.camera_path(s.cam, 6, step=7.0, yaw_step_deg=0.2)
    prev_cas, prev_tex = None, None
    total = 0
    for f, cam in enumerate(path):
        cas = _fit(s, cam)
        reused = gpu.zeros(1, dtype=gpu.int32, device="cuda")
        if prev_cas is None:
            tex = api.discretize(L, s.dom, cas)
        else:
            tex = api.discretize_reuse(L, s.dom, cas, prev_cas, prev_tex, reused=reused)
        t = tex.cpu().numpy()
        _check_oracle(s, cas, t)
        total += int(reused.item())
        prev_cas, prev_tex = cas, tex
    assert total > 0


def test_same_frame_copies_every_visible_block(gpu, tiny_scene, L):
    s = tiny_scene
    cas = _fit(s, s.cam)
    first = api.discretize(L, s.dom, cas)
    reused = gpu.zeros(1, dtype=gpu.int32, device="cuda")
    again = api.discretize_reuse(L, s.dom, cas, cas, first, reused=reused)
    assert gpu.equal(again, first)
    t = first.cpu().numpy()
    K, N = t.shape[0], t.shape[1]
    nb = (N + 15) // 16
    pad = np.zeros((K, nb * 16, nb * 16), bool)
    pad[:, :N, :N] = np.isfinite(t)
    blocks = int(pad.reshape(K, nb, 16, nb, 16).any(axis=(2, 4)).sum())
    assert int(reused.item()) == blocks


def test_shifted_lattice_and_foreign_spacing(gpu, tiny_scene, L):
    s = tiny_scene
    cas = _fit(s, s.cam)
    K = len(cas)
    # the previous frame: the same cascades moved by whole texels (5 right, 3 down)
    prev = (api.Cascade * K)()
    for k in range(K):
        prev[k] = cas[k]
        prev[k].x0 = cas[k].x0 - 5 * cas[k].hx
        prev[k].y0 = cas[k].y0 + 3 * cas[k].hy
    prev_tex = api.discretize(L, s.dom, prev)
    reused = gpu.zeros(1, dtype=gpu.int32, device="cuda")
    tex = api.discretize_reuse(L, s.dom, cas, prev, prev_tex, reused=reused)
    assert int(reused.item()) > 0
    t = tex.cpu().numpy()
    _check_oracle(s, cas, t)
    # texel (i, j) now is texel (i + 5, j - 3) then; copied blocks hold those values bit for bit
    p = prev_tex.cpu().numpy()
    N = t.shape[1]
    a, b = t[:, 3:, :N - 5], p[:, :N - 3, 5:]
    same = np.isfinite(a) & np.isfinite(b)
    assert np.count_nonzero(a[same] == b[same]) >= 0.5 * same.sum()
    # another spacing: nothing copied, the plain result
    for k in range(K):
        prev[k].hx = cas[k].hx * 1.189207115002721
    reused.zero_()
    tex2 = api.discretize_reuse(L, s.dom, cas, prev, prev_tex, reused=reused)
    assert int(reused.item()) == 0
    assert gpu.equal(tex2, api.discretize(L, s.dom, cas))


def test_renderer_flight_matches_fresh_frames(gpu, tiny_scene):
    from paper_2201_10887_amd.renderer import Renderer
    s = tiny_scene
    w = s.work
    args = (dict(s.leaves), w.side, w.max_depth, w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    Rr, Rf = Renderer(*args), Renderer(*args)
    Rr.set_texel_reuse(True)
    Rr.count_reused = True
    Rr.reused_blocks.zero_()
    for cam in synth.camera_path(s.cam, 5, step=9.0):
        dr, hr, cr = Rr.forward(cam)
        df, hf, _ = Rf.forward(cam, cascades=cr)  # the same fixed-lattice cascades, every texel computed
        a, b = Rr.tex.cpu().numpy(), Rf.tex.cpu().numpy()
        assert np.array_equal(np.isfinite(a), np.isfinite(b))
        fin = np.isfinite(b)
        assert np.all(np.abs(a[fin] - b[fin]) <= G.texel_tolerance(s.leaves, b[fin]))
        dr, df = dr.cpu().numpy(), df.cpu().numpy()
        both = np.isfinite(dr) & np.isfinite(df)
        diff = np.zeros_like(dr)
        diff[both] = dr[both] - df[both]
        bad = (np.isfinite(dr) != np.isfinite(df)) | (np.abs(diff) > 1e-4 * s.dom.extent)
        assert bad.mean() <= 1e-3, bad.sum()
    assert int(Rr.reused_blocks.item()) > 0


def test_renderer_flight_with_water_matches_fresh_frames(gpu, tiny_scene):
    """Reuse with two surfaces: each surface keeps its own pair of texture buffers."""
    from paper_2201_10887_amd.renderer import Renderer
    s = tiny_scene
    w = s.work
    args = (dict(s.leaves), w.side, w.max_depth, w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    water = synth.water_surface(s.leaves, w.side, 91)
    Rr, Rf = Renderer(*args), Renderer(*args)
    for R in (Rr, Rf):
        R.add_surface(water)
    Rr.set_texel_reuse(True)
    Rr.count_reused = True
    Rr.reused_blocks.zero_()
    for cam in synth.camera_path(s.cam, 4, step=9.0):
        dr, hr, cr = Rr.forward(cam)
        df, hf, _ = Rf.forward(cam, cascades=cr)
        for (_, tr, _, _), (_, tf, _, _) in zip(Rr.surfaces(), Rf.surfaces()):
            a, b = tr.cpu().numpy(), tf.cpu().numpy()
            assert np.array_equal(np.isfinite(a), np.isfinite(b))
            fin = np.isfinite(b)
            assert np.all(np.abs(a[fin] - b[fin]) <= G.texel_tolerance(s.leaves, b[fin]) + 1e-5 * np.abs(water).max())
        dr, df = dr.cpu().numpy(), df.cpu().numpy()
        both = np.isfinite(dr) & np.isfinite(df)
        diff = np.zeros_like(dr)
        diff[both] = dr[both] - df[both]
        bad = (np.isfinite(dr) != np.isfinite(df)) | (np.abs(diff) > 1e-4 * s.dom.extent)
        assert bad.mean() <= 1e-3, bad.sum()
    assert int(Rr.reused_blocks.item()) > 0
