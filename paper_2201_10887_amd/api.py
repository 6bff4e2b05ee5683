"""Python binding of libhfr with the C ABI's names (argument marshalling only).

Host entry points take and return NumPy arrays; device entry points take
torch CUDA tensors (ROCm) and enqueue on torch's current stream unless a
stream is given.  Every computation runs in libhfr; this module only checks
shapes and dtypes and converts structures.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import Camera, Cascade, Domain, Leaves, call


# ------------------------------------------------------------------ helpers

def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _dev(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def camera(cam) -> Camera:
    c = Camera()
    c.pos[:] = [float(v) for v in cam.pos]
    c.yaw, c.pitch, c.vfov = float(cam.yaw), float(cam.pitch), float(cam.vfov)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(getattr(cam, "znear", 1.0))
    return c


def domain(dom) -> Domain:
    return Domain(float(dom.x0), float(dom.y0), float(dom.x1), float(dom.y1), float(dom.zmin), float(dom.zmax))


def cascades_from(objs: Sequence) -> ctypes.Array:
    """Pack cascade descriptions (objects with near/far/split/origin/vhat/x0/y0/hx/hy/n/poly) for the ABI."""
    arr = (Cascade * len(objs))()
    for a, o in enumerate(objs):
        c = arr[a]
        c.near_d, c.far_d, c.split_d = float(o.near), float(o.far), float(o.split)
        c.origin[:] = [float(o.origin[0]), float(o.origin[1])]
        c.vhat[:] = [float(o.vhat[0]), float(o.vhat[1])]
        c.x0, c.y0, c.hx, c.hy = float(o.x0), float(o.y0), float(o.hx), float(o.hy)
        c.n = int(o.n)
        poly = np.asarray(o.poly, np.float64).reshape(-1, 2)
        if len(poly) > _lib.HFR_MAX_POLY:
            raise ValueError("cascade polygon has too many vertices")
        c.n_poly = len(poly)
        for v in range(len(poly)):
            c.poly[v][0], c.poly[v][1] = float(poly[v, 0]), float(poly[v, 1])
    return arr


class CascadeView:
    """Read-only attribute view of one ABI cascade (same field names as the oracle's)."""

    def __init__(self, c: Cascade):
        self.near, self.far, self.split = c.near_d, c.far_d, c.split_d
        self.origin = np.array(c.origin[:])
        self.vhat = np.array(c.vhat[:])
        self.x0, self.y0, self.hx, self.hy, self.n = c.x0, c.y0, c.hx, c.hy, c.n
        self.poly = np.array([[c.poly[v][0], c.poly[v][1]] for v in range(c.n_poly)]).reshape(-1, 2)


# ------------------------------------------------------------- start-up (host)

def abi_version() -> int:
    return _lib.load().hfr_abi_version()


def runtime_version() -> int:
    v = ctypes.c_int(0)
    call("hfr_runtime_version", ctypes.byref(v))
    return v.value


def build_quadtree(dem: np.ndarray, side: float, max_depth: int, tau: float, x0: float = 0.0,
                   y0: float = 0.0) -> dict:
    dem = np.ascontiguousarray(dem, np.float32)
    if dem.ndim != 2 or dem.shape[0] != dem.shape[1]:
        raise ValueError("raster must be square")
    q = ctypes.c_void_p()
    call("hfr_build_quadtree", _np_ptr(dem), dem.shape[0], side, x0, y0, max_depth, tau, ctypes.byref(q))
    lib = _lib.load()
    try:
        n = ctypes.c_int64()
        call("hfr_quadtree_size", q, ctypes.byref(n))
        out = {k: np.empty(n.value, np.float32) for k in ("x", "y", "c", "v")}
        out.update({k: np.empty(n.value, np.int32) for k in ("level", "i", "j")})
        call("hfr_quadtree_export", q, *(_np_ptr(out[k]) for k in ("x", "y", "c", "v", "level", "i", "j")))
    finally:
        lib.hfr_quadtree_destroy(q)
    return out


def build_quadtree_device(dem, side: float, max_depth: int, tau: float, x0: float = 0.0, y0: float = 0.0,
                          stream=None) -> dict:
    """The quadtree built on the device from a device raster (torch tensor, float32 [n][n]).

    Returns device tensors ``x, y, c, v`` (float32) and ``level, i, j`` (int32), sorted by (level, row,
    column), with their level index ``rank`` and ``order`` (0 .. n-1): ``(rank, order)`` is what
    ``DeviceLeaves.from_device`` takes."""
    import torch
    n = int(dem.shape[0])
    if dem.dim() != 2 or dem.shape[1] != n:
        raise ValueError("raster must be square")
    _dev(dem, torch.float32, (n, n), "dem")
    nbytes = ctypes.c_int64()
    call("hfr_quadtree_device_workspace", n, max_depth, ctypes.byref(nbytes))
    work = torch.empty(nbytes.value, dtype=torch.uint8, device=dem.device)
    rank = torch.empty(rank_table_size(max_depth), dtype=torch.int32, device=dem.device)
    count = ctypes.c_int64()
    call("hfr_build_quadtree_device", dem.data_ptr(), n, side, x0, y0, max_depth, tau, work.data_ptr(),
         rank.data_ptr(), ctypes.byref(count), _stream(stream))
    m = count.value
    out = {k: torch.empty(m, dtype=torch.float32, device=dem.device) for k in ("x", "y", "c", "v")}
    out.update({k: torch.empty(m, dtype=torch.int32, device=dem.device) for k in ("level", "i", "j")})
    call("hfr_quadtree_device_leaves", n, side, x0, y0, max_depth, work.data_ptr(), rank.data_ptr(), m,
         *(out[k].data_ptr() for k in ("x", "y", "c", "v", "level", "i", "j")), _stream(stream))
    out["rank"] = rank
    out["order"] = torch.arange(m, dtype=torch.int32, device=dem.device)
    return out


def build_neighbours_device(L: "DeviceLeaves", slack: float = 1e-3, stream=None) -> tuple:
    """``build_neighbours`` on the device for packed ``DeviceLeaves`` (level radii written): device
    tensors ``(off int64[n + 1], idx int32[nnz])`` indexed by sorted position (leaf indices for leaves
    from ``build_quadtree_device``)."""
    import torch
    dev = L.x.device
    nbytes = ctypes.c_int64()
    call("hfr_neighbours_device_workspace", L.n, ctypes.byref(nbytes))
    work = torch.empty(max(nbytes.value, 8), dtype=torch.uint8, device=dev)
    off = torch.empty(L.n + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64()
    Ls = L.struct()
    call("hfr_build_neighbours_device", ctypes.byref(Ls), slack, work.data_ptr(), off.data_ptr(), ctypes.byref(nnz),
         _stream(stream))
    idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    call("hfr_neighbours_device_fill", ctypes.byref(Ls), slack, off.data_ptr(), idx.data_ptr(), _stream(stream))
    return off, idx[:nnz.value]


def quadtree_leaf_count(dem: np.ndarray, side: float, max_depth: int, tau: float) -> int:
    """Leaf count of ``build_quadtree`` without exporting the leaves."""
    dem = np.ascontiguousarray(dem, np.float32)
    q = ctypes.c_void_p()
    call("hfr_build_quadtree", _np_ptr(dem), dem.shape[0], side, 0.0, 0.0, max_depth, tau, ctypes.byref(q))
    try:
        n = ctypes.c_int64()
        call("hfr_quadtree_size", q, ctypes.byref(n))
        return int(n.value)
    finally:
        _lib.load().hfr_quadtree_destroy(q)


def build_neighbours(leaves: dict, side: float, max_depth: int, cutoff: float, slack: float = 1e-3,
                     x0: float = 0.0, y0: float = 0.0) -> tuple:
    arrs = [np.ascontiguousarray(leaves[k], np.float32) for k in ("x", "y", "c", "sigma")]
    n = len(arrs[0])
    h = ctypes.c_void_p()
    call("hfr_build_neighbours", n, *(_np_ptr(a) for a in arrs), x0, y0, side, max_depth, cutoff, slack,
         ctypes.byref(h))
    lib = _lib.load()
    try:
        nnz = ctypes.c_int64()
        call("hfr_neighbours_size", h, ctypes.byref(nnz))
        off = np.empty(n + 1, np.int32)
        idx = np.empty(max(nnz.value, 1), np.int32)[:nnz.value]
        call("hfr_neighbours_export", h, _np_ptr(off), _np_ptr(idx))
    finally:
        lib.hfr_neighbours_destroy(h)
    return off, idx


def rank_table_size(max_depth: int) -> int:
    return ((1 << (2 * (max_depth + 1))) - 1) // 3 + max_depth + 1


def rank_offset(level: int) -> int:
    """Offset of a level's 4^level + 1 prefix counts in the rank table."""
    return ((1 << (2 * level)) - 1) // 3 + level


def build_level_index(leaves: dict, side: float, max_depth: int, x0: float = 0.0, y0: float = 0.0):
    """``(rank, order)``: the leaves sorted by (level, row, column) and per-level prefix counts."""
    arrs = [np.ascontiguousarray(leaves[k], np.float32) for k in ("x", "y", "c")]
    rank = np.empty(rank_table_size(max_depth), np.int32)
    order = np.empty(len(arrs[0]), np.int32)
    call("hfr_build_level_index", len(arrs[0]), *(_np_ptr(a) for a in arrs), x0, y0, side, max_depth,
         _np_ptr(rank), _np_ptr(order))
    return rank, order


def fit_cascades(cam, dom, K: int, N: int, lam: float, overlap: float, c_min: float,
                 aligned: bool = False) -> ctypes.Array:
    """Cascades of one camera; ``aligned``: texel lattices fixed in the world (hfr_fit_cascades_aligned)."""
    out = (Cascade * K)()
    call("hfr_fit_cascades_aligned" if aligned else "hfr_fit_cascades", ctypes.byref(camera(cam)),
         ctypes.byref(domain(dom)), K, N, lam, overlap, c_min, out)
    return out


# ---------------------------------------------------------- per frame (device)

BASIS_GAUSSIAN = 0  # Eq. 1
BASIS_WENDLAND = 1  # Wendland's C2 function on the same support
BASES = {"gaussian": BASIS_GAUSSIAN, "wendland": BASIS_WENDLAND}


class DeviceLeaves:
    """Leaf arrays, level index and per-level radii resident on the GPU (torch tensors).  ``basis``
    (``BASIS_*``) is the weight function the packed records are written for."""

    def __init__(self, leaves: dict, index, side: float, max_depth: int, cutoff: float,
                 x0: float = 0.0, y0: float = 0.0, device: str = "cuda"):
        import torch
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
        self.x, self.y, self.c = f(leaves["x"]), f(leaves["y"]), f(leaves["c"])
        self.v, self.sigma = f(leaves["v"]), f(leaves["sigma"])
        rank, order = index
        if len(rank) != rank_table_size(max_depth) or len(order) != len(leaves["x"]):
            raise ValueError("level index does not match max_depth and the leaf count")
        self.rank = torch.as_tensor(np.ascontiguousarray(rank, np.int32), device=device)
        self.order = torch.as_tensor(np.ascontiguousarray(order, np.int32), device=device)
        self.n = len(leaves["x"])
        self.packed = torch.empty((self.n, 4), dtype=torch.float32, device=device)
        self.level_radius = torch.zeros(max_depth + 1, dtype=torch.float32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.max_depth, self.cutoff = int(max_depth), float(cutoff)
        self.x0, self.y0, self.side = float(x0), float(y0), float(side)
        self.basis = BASIS_GAUSSIAN

    @classmethod
    def from_device(cls, leaves: dict, sigma, side: float, max_depth: int, cutoff: float, x0: float = 0.0,
                    y0: float = 0.0) -> "DeviceLeaves":
        """From ``build_quadtree_device`` output (device tensors, level index included) and widths
        ``sigma`` (a device tensor or a scalar); nothing goes through the host."""
        import torch
        self = object.__new__(cls)
        dev = leaves["x"].device
        self.x, self.y, self.c, self.v = (leaves[k].contiguous() for k in ("x", "y", "c", "v"))
        self.n = int(self.x.numel())
        self.sigma = (sigma.to(dev, torch.float32).contiguous() if torch.is_tensor(sigma)
                      else torch.full((self.n,), float(sigma), dtype=torch.float32, device=dev))
        self.rank, self.order = leaves["rank"], leaves["order"]
        if self.rank.numel() != rank_table_size(max_depth):
            raise ValueError("level index does not match max_depth")
        self.packed = torch.empty((self.n, 4), dtype=torch.float32, device=dev)
        self.level_radius = torch.zeros(max_depth + 1, dtype=torch.float32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.max_depth, self.cutoff = int(max_depth), float(cutoff)
        self.x0, self.y0, self.side = float(x0), float(y0), float(side)
        self.basis = BASIS_GAUSSIAN
        return self

    def with_values(self, v) -> "DeviceLeaves":
        """Another heightfield on the same cells (shares positions, sizes, widths and the level index):
        values ``v``, its own packed records and level radii (call ``pack_leaves`` on it)."""
        import torch
        other = object.__new__(DeviceLeaves)
        other.__dict__.update(self.__dict__)
        other.v = torch.as_tensor(np.ascontiguousarray(v, np.float32), device=self.x.device)
        if other.v.numel() != self.n:
            raise ValueError("one value per leaf is required")
        other.packed = torch.empty_like(self.packed)
        other.level_radius = torch.zeros_like(self.level_radius)
        other.status = torch.zeros_like(self.status)
        return other

    def with_basis(self, basis) -> "DeviceLeaves":
        """The same heightfield reconstructed with another weight function (``BASIS_*`` or its name):
        shares every leaf array and the level index; its own packed records (call ``pack_leaves``)."""
        import torch
        b = BASES[basis] if isinstance(basis, str) else int(basis)
        if b not in BASES.values():
            raise ValueError(f"unknown basis {basis!r}")
        other = object.__new__(DeviceLeaves)
        other.__dict__.update(self.__dict__)
        other.basis = b
        other.packed = torch.empty_like(self.packed)
        other.level_radius = torch.zeros_like(self.level_radius)
        other.status = torch.zeros_like(self.status)
        return other

    def struct(self) -> Leaves:
        import torch
        for name in ("x", "y", "c", "v", "sigma", "packed", "level_radius"):
            _dev(getattr(self, name), torch.float32, None, name)
        _dev(self.rank, torch.int32, None, "rank")
        _dev(self.order, torch.int32, (self.n,), "order")
        _dev(self.status, torch.int32, (1,), "status")
        return Leaves(self.n, self.x.data_ptr(), self.y.data_ptr(), self.c.data_ptr(), self.v.data_ptr(),
                      self.sigma.data_ptr(), self.packed.data_ptr(), self.level_radius.data_ptr(),
                      self.rank.data_ptr(), self.order.data_ptr(), self.max_depth, self.cutoff, self.x0, self.y0,
                      self.side, self.basis, self.status.data_ptr())


def pack_leaves(L: DeviceLeaves, stream=None, check: bool = True) -> None:
    """``hfr_pack_leaves``; with ``check`` the leaves' status word is read back (one synchronisation)
    and a refusal raised as ``HfrError``."""
    call("hfr_pack_leaves", ctypes.byref(L.struct()), _stream(stream))
    if check:
        leaf_status(L)


def leaf_status(L: DeviceLeaves) -> None:
    """Raise ``HfrError`` (HFR_EINVAL) if the last ``pack_leaves`` refused the leaves (reads the device
    status word: synchronises with its stream)."""
    st = int(L.status.item())
    if st != 0:
        raise _lib.HfrError("hfr_pack_leaves", st, f"a leaf has cutoff * sigma <= sqrt(2)/2 (cutoff {L.cutoff}) "
                                                    "or a non-finite value or width")


def discretize(L: DeviceLeaves, dom, cascades: ctypes.Array, tex=None, mask=None, stream=None):
    import torch
    K, N = len(cascades), cascades[0].n
    if tex is None:
        tex = torch.empty((K, N, N), dtype=torch.float32, device=L.x.device)
    tp = _dev(tex, torch.float32, (K, N, N), "tex")
    mp = _dev(mask, torch.int32, (K, N, (N + 31) // 32), "mask") if mask is not None else None
    call("hfr_discretize", ctypes.byref(L.struct()), ctypes.byref(domain(dom)), cascades, K, tp, mp,
         _stream(stream))
    return tex


def discretize_reuse(L: DeviceLeaves, dom, cascades: ctypes.Array, prev_cascades: ctypes.Array, prev_tex, tex=None,
                     mask=None, reused=None, stream=None):
    """``discretize`` for the next frame, copying the blocks whose texels the previous frame already
    holds (``prev_cascades``, ``prev_tex``; same leaves).  ``reused``: int32 device tensor [1] that
    counts the copied 16 x 16 blocks (caller-zeroed), or None."""
    import torch
    K, N = len(cascades), cascades[0].n
    if len(prev_cascades) != K:
        raise ValueError("prev_cascades must hold one cascade per cascade")
    if tex is None:
        tex = torch.empty((K, N, N), dtype=torch.float32, device=L.x.device)
    tp = _dev(tex, torch.float32, (K, N, N), "tex")
    pp = _dev(prev_tex, torch.float32, (K, N, N), "prev_tex")
    mp = _dev(mask, torch.int32, (K, N, (N + 31) // 32), "mask") if mask is not None else None
    rp = _dev(reused, torch.int32, (1,), "reused") if reused is not None else None
    call("hfr_discretize_reuse", ctypes.byref(L.struct()), ctypes.byref(domain(dom)), cascades, K, prev_cascades, pp,
         tp, mp, rp, _stream(stream))
    return tex


def mip_size(N: int) -> int:
    return (4 * N * N - 1) // 3


def build_maxmip(tex, mip=None, stream=None):
    import torch
    K, N = tex.shape[0], tex.shape[1]
    if mip is None:
        mip = torch.empty((K, mip_size(N)), dtype=torch.float32, device=tex.device)
    call("hfr_build_maxmip", _dev(tex, torch.float32, (K, N, N), "tex"), K, N,
         _dev(mip, torch.float32, (K, mip_size(N)), "mip"), _stream(stream))
    return mip


def ray_workspace(cam, device) -> "torch.Tensor":
    """Scratch for the long-ray queue of ``raycast`` / ``raycast_backward`` (int32[W H + 2])."""
    import torch
    return torch.empty(cam.width * cam.height + 2, dtype=torch.int32, device=device)


def _work_ptr(work, cam, device):
    """``work``: a workspace tensor, True (allocate one) or None / False (no long-ray queue)."""
    import torch
    if work is None or work is False:
        return None
    if work is True:
        work = ray_workspace(cam, device)
    return _dev(work, torch.int32, (cam.width * cam.height + 2,), "work")


def raycast(cam, dom, cascades: ctypes.Array, tex, mip, depth=None, hit=None, stream=None, work=True,
            band_rows=None):
    """``hfr_raycast``; with ``band_rows`` (and a workspace) ``hfr_raycast_split``."""
    import torch
    K, N = len(cascades), cascades[0].n
    if depth is None:
        depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device=tex.device)
    if hit is None:
        hit = torch.empty((cam.height, cam.width), dtype=torch.int32, device=tex.device)
    args = [ctypes.byref(camera(cam)), ctypes.byref(domain(dom)), cascades, K,
            _dev(tex, torch.float32, (K, N, N), "tex"), _dev(mip, torch.float32, (K, mip_size(N)), "mip"),
            _dev(depth, torch.float32, (cam.height, cam.width), "depth"),
            _dev(hit, torch.int32, (cam.height, cam.width), "hit"), _work_ptr(work, cam, tex.device)]
    if band_rows is None:
        call("hfr_raycast", *args, _stream(stream))
    else:
        call("hfr_raycast_split", *args, int(band_rows), _stream(stream))
    return depth, hit


def band_rows(cam, degrees: float) -> int:
    """Image rows whose central ray points at most ``degrees`` below the horizontal (the camera has no
    roll, so a row's elevation is pitch + atan(s tan(vfov / 2)), s from 1 at the top to -1 at the bottom);
    the band ``raycast(..., band_rows=)`` walks first."""
    ty = math.tan(0.5 * cam.vfov)
    a = min(max(-math.radians(degrees) - cam.pitch, -1.55), 1.55)
    s = math.tan(a) / ty  # rows with s >= this are in the band
    rows = int(math.floor(0.5 * cam.height * (1.0 - s)))
    return min(max(rows, 0), cam.height)


def raycast_static_max_pixels() -> int:
    n = ctypes.c_int64()
    call("hfr_raycast_static_max_pixels", ctypes.byref(n))
    return n.value


def raycast_static(cam, dom, cascades: ctypes.Array, tex, mip, depth, hit, stream=None):
    """``raycast`` with the long-ray queue in the library's static device array (allocates nothing;
    ``depth`` and ``hit`` are required)."""
    import torch
    K, N = len(cascades), cascades[0].n
    call("hfr_raycast_static", ctypes.byref(camera(cam)), ctypes.byref(domain(dom)), cascades, K,
         _dev(tex, torch.float32, (K, N, N), "tex"), _dev(mip, torch.float32, (K, mip_size(N)), "mip"),
         _dev(depth, torch.float32, (cam.height, cam.width), "depth"),
         _dev(hit, torch.int32, (cam.height, cam.width), "hit"), _stream(stream))
    return depth, hit


def raycast_backward(cam, dom, cascades: ctypes.Array, tex, mip, grad_depth, grad_tex=None, stream=None,
                     work=True, band_rows=None):
    """``hfr_raycast_backward``; with ``band_rows`` (and a workspace) ``hfr_raycast_backward_split``."""
    import torch
    K, N = len(cascades), cascades[0].n
    if grad_tex is None:
        grad_tex = torch.zeros((K, N, N), dtype=torch.float32, device=tex.device)
    args = [ctypes.byref(camera(cam)), ctypes.byref(domain(dom)), cascades, K,
            _dev(tex, torch.float32, (K, N, N), "tex"), _dev(mip, torch.float32, (K, mip_size(N)), "mip"),
            _dev(grad_depth, torch.float32, (cam.height, cam.width), "grad_depth"),
            _dev(grad_tex, torch.float32, (K, N, N), "grad_tex"), _work_ptr(work, cam, tex.device)]
    if band_rows is None:
        call("hfr_raycast_backward", *args, _stream(stream))
    else:
        call("hfr_raycast_backward_split", *args, int(band_rows), _stream(stream))
    return grad_tex


def raycast_nearer(cam, dom, cascades: ctypes.Array, tex, mip, surface: int, depth, hit, stream=None, work=True):
    """Draw a further surface over ``depth`` / ``hit`` (in place) where it is nearer."""
    import torch
    K, N = len(cascades), cascades[0].n
    call("hfr_raycast_nearer", ctypes.byref(camera(cam)), ctypes.byref(domain(dom)), cascades, K,
         _dev(tex, torch.float32, (K, N, N), "tex"), _dev(mip, torch.float32, (K, mip_size(N)), "mip"), int(surface),
         _dev(depth, torch.float32, (cam.height, cam.width), "depth"),
         _dev(hit, torch.int32, (cam.height, cam.width), "hit"), _work_ptr(work, cam, tex.device), _stream(stream))
    return depth, hit


def raycast_backward_surface(cam, dom, cascades: ctypes.Array, tex, mip, surface: int, hit, grad_depth,
                             grad_tex=None, stream=None, work=True):
    """Texel gradients of surface ``surface`` over the pixels whose final hit it is."""
    import torch
    K, N = len(cascades), cascades[0].n
    if grad_tex is None:
        grad_tex = torch.zeros((K, N, N), dtype=torch.float32, device=tex.device)
    call("hfr_raycast_backward_surface", ctypes.byref(camera(cam)), ctypes.byref(domain(dom)), cascades, K,
         _dev(tex, torch.float32, (K, N, N), "tex"), _dev(mip, torch.float32, (K, mip_size(N)), "mip"), int(surface),
         _dev(hit, torch.int32, (cam.height, cam.width), "hit"),
         _dev(grad_depth, torch.float32, (cam.height, cam.width), "grad_depth"),
         _dev(grad_tex, torch.float32, (K, N, N), "grad_tex"), _work_ptr(work, cam, tex.device), _stream(stream))
    return grad_tex


def discretize_backward(L: DeviceLeaves, dom, cascades: ctypes.Array, tex, grad_tex, grad_v=None,
                        grad_sigma=None, stream=None):
    import torch
    K, N = len(cascades), cascades[0].n
    if grad_v is None:
        grad_v = torch.zeros(L.n, dtype=torch.float32, device=tex.device)
    if grad_sigma is None:
        grad_sigma = torch.zeros(L.n, dtype=torch.float32, device=tex.device)
    call("hfr_discretize_backward", ctypes.byref(L.struct()), ctypes.byref(domain(dom)), cascades, K,
         _dev(tex, torch.float32, (K, N, N), "tex"), _dev(grad_tex, torch.float32, (K, N, N), "grad_tex"),
         _dev(grad_v, torch.float32, (L.n,), "grad_v"), _dev(grad_sigma, torch.float32, (L.n,), "grad_sigma"),
         _stream(stream))
    return grad_v, grad_sigma


# ------------------------------------------------------------------ batching

class BatchPlan:
    """Handle of an ``hfr_batch_plan`` plus references to every tensor it names
    (the plan stores raw device pointers, so the tensors must stay alive)."""

    def __init__(self, handle: ctypes.c_void_p, keep: list, n_views: int, ks: list):
        self.handle, self._keep, self.n_views, self.ks = handle, keep, n_views, ks

    def __del__(self):
        batch_plan_destroy(self)


def batch_plan_create(fields: Sequence[dict], views: Sequence[dict]) -> BatchPlan:
    """``fields``: dicts with ``leaves`` (DeviceLeaves), ``dom`` and optional ``grad_v`` /
    ``grad_sigma`` (float32 [n]).  ``views``: dicts with ``field, K, N, width, height,
    split_lambda, overlap, c_min, tex, mip, depth, hit`` and optional ``mask, grad_depth,
    grad_tex`` (shapes as for the per-view entry points)."""
    import torch
    keep = []
    farr = (_lib.BatchField * len(fields))()
    for a, f in enumerate(fields):
        L = f["leaves"]
        farr[a].leaves = L.struct()
        farr[a].dom = domain(f["dom"])
        for name in ("grad_v", "grad_sigma"):
            t = f.get(name)
            setattr(farr[a], name, _dev(t, torch.float32, (L.n,), name).value if t is not None else None)
            keep.append(t)
        keep.append(L)
    varr = (_lib.BatchView * len(views))()
    for a, v in enumerate(views):
        K, N, W, H = int(v["K"]), int(v["N"]), int(v["width"]), int(v["height"])
        b = varr[a]
        b.field, b.K, b.N, b.width, b.height = int(v["field"]), K, N, W, H
        b.split_lambda, b.overlap, b.c_min = float(v["split_lambda"]), float(v["overlap"]), float(v["c_min"])
        b.tex = _dev(v["tex"], torch.float32, (K, N, N), "tex").value
        b.mip = _dev(v["mip"], torch.float32, (K, mip_size(N)), "mip").value
        b.depth = _dev(v["depth"], torch.float32, (H, W), "depth").value
        b.hit = _dev(v["hit"], torch.int32, (H, W), "hit").value
        m, gd, gt = v.get("mask"), v.get("grad_depth"), v.get("grad_tex")
        b.mask = _dev(m, torch.int32, (K, N, (N + 31) // 32), "mask").value if m is not None else None
        b.grad_depth = _dev(gd, torch.float32, (H, W), "grad_depth").value if gd is not None else None
        b.grad_tex = _dev(gt, torch.float32, (K, N, N), "grad_tex").value if gt is not None else None
        keep.extend([v["tex"], v["mip"], v["depth"], v["hit"], m, gd, gt])
    handle = ctypes.c_void_p()
    call("hfr_batch_plan_create", farr, len(fields), varr, len(views), ctypes.byref(handle))
    return BatchPlan(handle, keep, len(views), [int(v["K"]) for v in views])


def batch_plan_destroy(plan: BatchPlan) -> None:
    if getattr(plan, "handle", None) is not None and plan.handle.value:
        _lib.load().hfr_batch_plan_destroy(plan.handle)
        plan.handle = None


def batch_set_tuning(plan: BatchPlan, disc_blocks_per_cu: int = 4, ray_blocks_per_cu: int = 4,
                     ray_tile_w: int = 32, disc_grain: int = 8, ray_queue: int = 0, ray_grain: int = 8) -> None:
    t = _lib.BatchTuning(int(disc_blocks_per_cu), int(ray_blocks_per_cu), int(ray_tile_w), int(disc_grain),
                         int(ray_queue), int(ray_grain))
    call("hfr_batch_set_tuning", plan.handle, ctypes.byref(t))


def batch_long_rays(plan: BatchPlan) -> np.ndarray:
    """Rays per view that the plan's last ray-cast launch sent to the long-ray queue (synchronises)."""
    out = np.zeros(plan.n_views, np.int32)
    call("hfr_batch_long_rays", plan.handle, out.ctypes.data_as(ctypes.c_void_p))
    return out


def batch_set_cameras(plan: BatchPlan, cams: Sequence, stream=None) -> None:
    arr = (Camera * len(cams))(*[camera(c) for c in cams])
    if len(cams) != plan.n_views:
        raise ValueError(f"{len(cams)} cameras for {plan.n_views} views")
    call("hfr_batch_set_cameras", plan.handle, arr, _stream(stream))


def batch_cascades(plan: BatchPlan, view: int) -> ctypes.Array:
    out = (Cascade * plan.ks[view])()
    call("hfr_batch_cascades", plan.handle, int(view), out)
    return out


def batch_launch(plan: BatchPlan, stream=None) -> None:
    call("hfr_batch_launch", plan.handle, _stream(stream))


def batch_launch_backward(plan: BatchPlan, stream=None) -> None:
    call("hfr_batch_launch_backward", plan.handle, _stream(stream))
