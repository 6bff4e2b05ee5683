"""hfr_raycast_static (the ray cast that allocates nothing) against hfr_raycast with a workspace.

Both calls run the same kernels; only the home of the long-ray queue differs
(the library's static device array instead of a caller tensor), so depth and
hit images must be identical.  Two calls in a row on one device, the second
with a smaller image, exercise the shared array: the second call must not
see the first call's queue.  The scene is the medium terrain (3.97M leaves,
4 x 2048^2 cascades), whose 1080p frame queues thousands of long rays.
"""
import numpy as np
import pytest

from paper_2201_10887_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frame():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = synth.MEDIUM
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed)
    leaves = api.build_quadtree(dem, w.side, w.max_depth, w.tau)
    leaves["sigma"] = np.full(len(leaves["x"]), w.sigma, np.float32)
    index = api.build_level_index(leaves, w.side, w.max_depth)
    L = api.DeviceLeaves(leaves, index, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(L)
    dom = synth.Domain(0.0, 0.0, w.side, w.side, float(leaves["v"].min()), float(leaves["v"].max()))
    cam = synth.camera_of(w, dem)
    cas = api.fit_cascades(cam, dom, w.cascades, w.tex_n, w.split_lambda, w.overlap, float(leaves["c"].min()))
    tex = api.discretize(L, dom, cas)
    mip = api.build_maxmip(tex)
    torch.cuda.synchronize()
    return dict(torch=torch, w=w, dem=dem, dom=dom, cam=cam, cas=cas, tex=tex, mip=mip, L=L, c_min=float(leaves["c"].min()))


def _with_workspace(f, cam, cas):
    torch = f["torch"]
    work = api.ray_workspace(cam, "cuda")
    depth, hit = api.raycast(cam, f["dom"], cas, f["tex"], f["mip"], work=work)
    torch.cuda.synchronize()
    return depth.cpu().numpy(), hit.cpu().numpy(), int(work[0].item())


def _static(f, cam, cas):
    torch = f["torch"]
    depth = torch.full((cam.height, cam.width), 7.0, dtype=torch.float32, device="cuda")
    hit = torch.full((cam.height, cam.width), 7, dtype=torch.int32, device="cuda")
    api.raycast_static(cam, f["dom"], cas, f["tex"], f["mip"], depth, hit)
    torch.cuda.synchronize()
    return depth.cpu().numpy(), hit.cpu().numpy()


def test_static_queue_equals_workspace_twice(frame):
    f = frame
    print("raycast_static: 1920x1080 then 640x360, medium scene", flush=True)
    cam1 = f["cam"]
    d_ref, h_ref, queued = _with_workspace(f, cam1, f["cas"])
    assert queued > 1000, queued  # the long-ray queue is in use on this frame
    d, h = _static(f, cam1, f["cas"])
    assert np.array_equal(h, h_ref)
    assert np.array_equal(d, d_ref, equal_nan=True)
    # a smaller image from a turned camera: the array keeps the first call's queue, which the
    # second call must clear before use
    cam2 = synth.Camera(tuple(cam1.pos), cam1.yaw + 0.3, cam1.pitch - 0.02, cam1.vfov, 640, 360, cam1.znear)
    w = f["w"]
    cas2 = api.fit_cascades(cam2, f["dom"], w.cascades, w.tex_n, w.split_lambda, w.overlap, f["c_min"])
    tex2 = api.discretize(f["L"], f["dom"], cas2)
    f2 = dict(f, tex=tex2, mip=api.build_maxmip(tex2))
    d_ref2, h_ref2, queued2 = _with_workspace(f2, cam2, cas2)
    d2, h2 = _static(f2, cam2, cas2)
    assert queued2 > 0, queued2
    assert np.array_equal(h2, h_ref2)
    assert np.array_equal(d2, d_ref2, equal_nan=True)


def test_static_queue_rejects_images_beyond_its_size(frame):
    f = frame
    torch = f["torch"]
    n = api.raycast_static_max_pixels()
    assert n == 1 << 22
    cam = synth.Camera(tuple(f["cam"].pos), f["cam"].yaw, f["cam"].pitch, f["cam"].vfov, 4096, 2048, f["cam"].znear)
    depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda")
    hit = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda")
    with pytest.raises(api._lib.HfrError) as e:
        api.raycast_static(cam, f["dom"], f["cas"], f["tex"], f["mip"], depth, hit)
    assert e.value.code == -1 and "static queue" in str(e.value)
