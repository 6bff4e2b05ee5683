"""Frame-level orchestration of the per-frame path on one GPU.

``Renderer`` owns the device-resident heightfield (leaves, level
index, per-level truncation radii) and the per-frame buffers (cascade textures,
visibility bits, max-mipmaps, and per image size the ray caster's long-ray
queue), all allocated once; ``forward`` runs cascade fitting (host),
discretize, max-mipmap and ray casting (device) on the current stream and
allocates nothing after the first frame of an image size.  ``RenderDepth`` is the
``torch.autograd.Function`` that takes an image loss back to leaf values and
Gaussian widths through the hand-written adjoints.
"""
from __future__ import annotations

import numpy as np

from . import api


class Renderer:
    def __init__(self, leaves: dict, side: float, max_depth: int, cutoff: float, cascades: int, tex_n: int,
                 split_lambda: float, overlap: float, device: str = "cuda",
                 x0: float = 0.0, y0: float = 0.0, basis="gaussian"):
        index = api.build_level_index(leaves, side, max_depth, x0, y0)
        L = api.DeviceLeaves(leaves, index, side, max_depth, cutoff, x0, y0, device=device)
        if basis != "gaussian":
            L = L.with_basis(basis)
        self._setup(L, float(np.min(leaves["c"])), float(np.min(leaves["v"])), float(np.max(leaves["v"])),
                    cascades, tex_n, split_lambda, overlap, device)

    @classmethod
    def from_raster(cls, dem, side: float, max_depth: int, tau: float, sigma, cutoff: float, cascades: int,
                    tex_n: int, split_lambda: float, overlap: float, x0: float = 0.0, y0: float = 0.0,
                    basis="gaussian") -> "Renderer":
        """The whole start-up on the device from a device raster (float32 [n][n] tensor): the quadtree
        and its level index (build_quadtree_device) and the packed records.  Only the leaf count, the
        smallest cell and the value range come back to the host.  ``sigma``: widths per leaf (tensor,
        in leaf order) or one width for all."""
        import torch
        q = api.build_quadtree_device(dem, side, max_depth, tau, x0, y0)
        L = api.DeviceLeaves.from_device(q, sigma, side, max_depth, cutoff, x0, y0)
        if basis != "gaussian":
            L = L.with_basis(basis)
        c_min, v_min, v_max = torch.stack([L.c.min(), L.v.min(), L.v.max()]).tolist()
        self = object.__new__(cls)
        self._setup(L, c_min, v_min, v_max, cascades, tex_n, split_lambda, overlap, str(dem.device))
        return self

    def _setup(self, L, c_min, v_min, v_max, cascades, tex_n, split_lambda, overlap, device):
        import torch
        self.side, self.max_depth, self.cutoff = L.side, L.max_depth, L.cutoff
        self.K, self.N, self.lam, self.overlap = int(cascades), int(tex_n), float(split_lambda), float(overlap)
        self.c_min = float(c_min)
        self.dom = api.domain(_Dom(L.x0, L.y0, L.x0 + L.side, L.y0 + L.side, float(v_min), float(v_max)))
        self.L = L
        api.pack_leaves(self.L)
        K, N = self.K, self.N
        self.tex = torch.empty((K, N, N), dtype=torch.float32, device=device)
        self.mask = torch.empty((K, N, (N + 31) // 32), dtype=torch.int32, device=device)
        self.mip = torch.empty((K, api.mip_size(N)), dtype=torch.float32, device=device)
        self.device = device
        # queue long rays for lane-shared walking (forward, adjoint); False: every ray finishes
        # on its own lane.  tune_raycast picks each by timing both on a camera.
        self.long_ray_queue = True
        self.long_ray_queue_backward = True
        # with the queue: split the frame at the row this many degrees below the horizon (rows above it
        # first, then their queued rays beside the rest); None: queue every row's long rays
        self.ray_band_deg = None
        self.ray_band_deg_backward = None
        self._work = {}
        self.extra = []  # further surfaces on the same cells (add_surface)
        # frame-to-frame texel reuse (set_texel_reuse): fixed-lattice cascades, a second texture set
        # per surface, the previous frame's cascades (None: nothing to reuse)
        self.texel_reuse = False
        self._spare = []
        self._prev_cas = None
        # count copied blocks into reused_blocks (one atomic per copied block on a single address:
        # measurable, so off unless asked for)
        self.count_reused = False
        self.reused_blocks = torch.zeros(1, dtype=torch.int32, device=device)
        # bumped by every call that rewrites textures or leaf records: an autograd node checks that
        # what its backward reads is still its own frame's
        self.generation = 0

    def ray_work(self, cam, backward: bool = False):
        """The long-ray queue for this camera's image size (None when disabled)."""
        if not (self.long_ray_queue_backward if backward else self.long_ray_queue):
            return None
        key = (cam.width, cam.height)
        if key not in self._work:
            self._work[key] = api.ray_workspace(cam, self.device)
        return self._work[key]

    def ray_band_rows(self, cam, backward: bool = False):
        """Rows walked before the queued long rays (None: no split), for this camera."""
        deg = self.ray_band_deg_backward if backward else self.ray_band_deg
        queue = self.long_ray_queue_backward if backward else self.long_ray_queue
        return api.band_rows(cam, deg) if (queue and deg is not None) else None

    def tune_raycast(self, cam, reps: int = 5, band_degrees=(3.0, 6.0, 12.0, 24.0)) -> dict:
        """Time the ray cast and its adjoint on this camera's frame every way the library offers and
        keep the fastest of each: each ray on its own lane, the long-ray queue after the whole frame,
        or the frame split at a row ``band_degrees`` below the horizon (the rows above first, then
        their queued rays beside the rest).  The queue pays off when a few long rays set the frame
        time; when the frame is throughput-bound, walking them after the rest costs more than it
        saves, and the split lets them run beside it.  Returns the median times (ms)."""
        import torch
        self.generation += 1
        cas = self.fit(cam)
        api.discretize(self.L, self.dom, cas, self.tex, self.mask)
        api.build_maxmip(self.tex, self.mip)
        depth = torch.empty((cam.height, cam.width), dtype=torch.float32, device=self.device)
        hit = torch.empty((cam.height, cam.width), dtype=torch.int32, device=self.device)
        work = api.ray_workspace(cam, self.device)
        api.raycast(cam, self.dom, cas, self.tex, self.mip, depth, hit, None, None)
        gd = torch.isfinite(depth).float()
        gtex = torch.zeros_like(self.tex)

        def median_ms(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b))
            return sorted(ts)[len(ts) // 2]

        res = {}
        ways = [("single_lane", None, None), ("queue", work, None)]
        ways += [(f"split_{d:g}deg", work, d) for d in band_degrees]
        for name, wk, deg in ways:
            band = None if deg is None else api.band_rows(cam, deg)
            res[f"raycast_{name}"] = median_ms(
                lambda: api.raycast(cam, self.dom, cas, self.tex, self.mip, depth, hit, None, wk, band))
            res[f"raycast_backward_{name}"] = median_ms(
                lambda: api.raycast_backward(cam, self.dom, cas, self.tex, self.mip, gd, gtex, None, wk, band))
        for prefix, attr_q, attr_d in (("raycast_", "long_ray_queue", "ray_band_deg"),
                                       ("raycast_backward_", "long_ray_queue_backward", "ray_band_deg_backward")):
            name, _, deg = min(ways, key=lambda w: res[prefix + w[0]])
            setattr(self, attr_q, name != "single_lane")
            setattr(self, attr_d, deg)
        self._work[(cam.width, cam.height)] = work
        return {k: round(v, 4) for k, v in res.items()}

    @property
    def domain(self):
        return self.dom

    def fit(self, cam):
        return api.fit_cascades(cam, self.dom, self.K, self.N, self.lam, self.overlap, self.c_min,
                                aligned=self.texel_reuse)

    def set_texel_reuse(self, on: bool = True):
        """Frame-to-frame texel reuse along a camera path: cascades fitted on lattices fixed in the world
        (``fit_cascades(..., aligned=True)``) and each frame's textures written into a second buffer,
        copying the 16 x 16 blocks the previous frame already holds (``discretize_reuse``).  Changing
        the leaves (``refresh_leaves``) or adding a surface forgets the previous frame."""
        import torch
        self.texel_reuse = bool(on)
        self._prev_cas = None
        self._spare = [torch.empty_like(tex) for _, tex, _, _ in self.surfaces()] if on else []

    def refresh_leaves(self, stream=None, check: bool = False):
        """Re-derive the packed leaf records after ``L.v`` or ``L.sigma`` changed (``check``: read back
        the leaves' status word and raise if a width is too small for Eq. 2; one synchronisation)."""
        self._prev_cas = None
        self.generation += 1
        api.pack_leaves(self.L, stream, check)
        for surf in self.extra:
            api.pack_leaves(surf["L"], stream, check)

    def add_surface(self, v) -> int:
        """A further heightfield on the same cells, e.g. terrain plus relative water depth (Section 2):
        values ``v`` per leaf, its own textures and pyramids over the same cascades, drawn where it is
        nearer.  Widens the domain's height range to cover it; returns the surface index."""
        import torch
        s = 1 + len(self.extra)
        if s >= 4:
            raise ValueError("at most four surfaces")
        self.generation += 1
        L = self.L.with_values(v)
        api.pack_leaves(L)
        d = self.dom
        self.dom = api.domain(_Dom(d.x0, d.y0, d.x1, d.y1, min(d.zmin, float(np.min(v))), max(d.zmax, float(np.max(v)))))
        K, N = self.K, self.N
        self._prev_cas = None
        if self.texel_reuse:
            self._spare.append(torch.empty_like(self.tex))
        self.extra.append({"L": L, "tex": torch.empty_like(self.tex), "mask": torch.empty_like(self.mask),
                           "mip": torch.empty_like(self.mip), "grad_tex": torch.zeros_like(self.tex),
                           "grad_v": torch.zeros(L.n, dtype=torch.float32, device=self.device)})
        return s

    def surfaces(self):
        """(leaves, textures, masks, pyramids) of every surface, surface 0 first."""
        yield self.L, self.tex, self.mask, self.mip
        for surf in self.extra:
            yield surf["L"], surf["tex"], surf["mask"], surf["mip"]

    def forward(self, cam, cascades=None, depth=None, hit=None, stream=None):
        self.generation += 1
        cas = self.fit(cam) if cascades is None else cascades
        for s, (L, tex, mask, mip) in enumerate(self.surfaces()):
            if self.texel_reuse and self._prev_cas is not None:
                new = self._spare[s]
                api.discretize_reuse(L, self.dom, cas, self._prev_cas, tex, new, mask,
                                     self.reused_blocks if self.count_reused else None, stream)
                self._spare[s] = tex
                if s == 0:
                    self.tex = new
                else:
                    self.extra[s - 1]["tex"] = new
                tex = new
            else:
                api.discretize(L, self.dom, cas, tex, mask, stream)
            api.build_maxmip(tex, mip, stream)
        if self.texel_reuse:
            self._prev_cas = cas
        work = self.ray_work(cam)
        depth, hit = api.raycast(cam, self.dom, cas, self.tex, self.mip, depth, hit, stream, work,
                                 self.ray_band_rows(cam) if work is not None else None)
        for s, surf in enumerate(self.extra, start=1):
            api.raycast_nearer(cam, self.dom, cas, surf["tex"], surf["mip"], s, depth, hit, stream, work)
        return depth, hit, cas

    def backward(self, cam, cascades, grad_depth, grad_tex, grad_v, grad_sigma, stream=None, hit=None,
                 surfaces=None):
        """Accumulates into the (caller-zeroed) gradient buffers.  With several surfaces, ``hit`` (the
        forward pass's) routes each pixel's gradient to the surface it shows: surface 0 into grad_tex and
        grad_v, surface s into its own zeroed ``extra[s - 1]["grad_tex"]`` / ``["grad_v"]``; the widths
        are shared, so grad_sigma sums over the surfaces.  ``surfaces``: (textures, pyramids) per surface
        to differentiate instead of the renderer's current ones (a kept copy of an earlier frame)."""
        work = self.ray_work(cam, backward=True)
        views = [(L, tex, mip) for L, tex, _, mip in self.surfaces()]
        if surfaces is not None:
            views = [(L, t, m) for (L, _, _), (t, m) in zip(views, surfaces)]
        if not self.extra:
            L, tex, mip = views[0]
            api.raycast_backward(cam, self.dom, cascades, tex, mip, grad_depth, grad_tex, stream, work,
                                 self.ray_band_rows(cam, backward=True) if work is not None else None)
            api.discretize_backward(L, self.dom, cascades, tex, grad_tex, grad_v, grad_sigma, stream)
            return grad_v, grad_sigma
        if hit is None:
            raise ValueError("several surfaces: pass the forward pass's hit buffer")
        for s, (L, tex, mip) in enumerate(views):
            gt = grad_tex if s == 0 else self.extra[s - 1]["grad_tex"]
            gv = grad_v if s == 0 else self.extra[s - 1]["grad_v"]
            if s > 0:
                gt.zero_()
                gv.zero_()
            api.raycast_backward_surface(cam, self.dom, cascades, tex, mip, s, hit, grad_depth, gt, stream, work)
            api.discretize_backward(L, self.dom, cascades, tex, gt, gv, grad_sigma, stream)
        return grad_v, grad_sigma


class _Dom:
    def __init__(self, x0, y0, x1, y1, zmin, zmax):
        self.x0, self.y0, self.x1, self.y1, self.zmin, self.zmax = x0, y0, x1, y1, zmin, zmax


def _make_function():
    import torch

    class RenderDepth(torch.autograd.Function):
        """depth = render(v, sigma, *water_values); backward gives d loss / d v, d loss / d sigma and,
        per further surface, d loss / d its values.

        The adjoints read the frame's textures, pyramids and leaf records.  By default they are the
        renderer's own buffers, so backward must come before the renderer draws again (it raises
        otherwise, instead of differentiating another frame).  ``snapshot=True`` keeps copies of this
        frame's textures, pyramids, values and widths, so several renders (e.g. two cameras) can be
        summed into one loss."""

        @staticmethod
        def forward(ctx, v, sigma, renderer: Renderer, cam, snapshot: bool, *extra_v):
            if len(extra_v) != len(renderer.extra):
                raise ValueError(f"the renderer has {len(renderer.extra)} further surfaces: pass one value "
                                 "tensor for each")
            L = renderer.L
            L.v.copy_(v.detach())
            L.sigma.copy_(sigma.detach())
            for surf, ev in zip(renderer.extra, extra_v):
                surf["L"].v.copy_(ev.detach())
            renderer.refresh_leaves()
            depth, hit, cas = renderer.forward(cam)
            ctx.renderer, ctx.cam, ctx.cas = renderer, cam, cas
            ctx.generation = renderer.generation
            ctx.snapshot = None
            if snapshot:
                ctx.snapshot = {"v": v.detach().clone(), "sigma": sigma.detach().clone(),
                                "extra_v": [e.detach().clone() for e in extra_v],
                                "surfaces": [(tex.clone(), mip.clone()) for _, tex, _, mip in renderer.surfaces()]}
            hit_out = hit.clone()
            ctx.hit = hit_out if renderer.extra else None
            ctx.mark_non_differentiable(hit_out)
            return depth.clone(), hit_out

        @staticmethod
        def backward(ctx, grad_depth, grad_hit):
            r = ctx.renderer
            surfaces = None
            if ctx.snapshot is not None:
                snap = ctx.snapshot
                if r.generation != ctx.generation:  # another frame was drawn since: restore this one's leaves
                    r.L.v.copy_(snap["v"])
                    r.L.sigma.copy_(snap["sigma"])
                    for surf, ev in zip(r.extra, snap["extra_v"]):
                        surf["L"].v.copy_(ev)
                    r.refresh_leaves()
                surfaces = snap["surfaces"]
            elif r.generation != ctx.generation:
                raise RuntimeError("render_depth: the renderer drew another frame (or changed its leaves) before "
                                   "this frame's backward; render with snapshot=True to sum several renders "
                                   "into one loss")
            gd = torch.where(torch.isfinite(grad_depth), grad_depth, torch.zeros_like(grad_depth)).contiguous()
            gtex = torch.zeros_like(r.tex)
            gv = torch.zeros(r.L.n, dtype=torch.float32, device=r.tex.device)
            gs = torch.zeros_like(gv)
            r.backward(ctx.cam, ctx.cas, gd, gtex, gv, gs, hit=ctx.hit, surfaces=surfaces)
            # each backward leaves its own frame's leaf records behind it
            extra_g = [surf["grad_v"].clone() for surf in r.extra]
            return (gv, gs, None, None, None, *extra_g)

    return RenderDepth


_RenderDepth = None


def render_depth(v, sigma, renderer: Renderer, cam, *extra_values, snapshot: bool = False):
    """Differentiable depth image (and non-differentiable hit ids) of leaf values ``v`` and widths
    ``sigma`` and, for a renderer with further surfaces, their values (one tensor per surface, each
    differentiable too).  ``snapshot``: keep this frame's textures so that the renderer may draw other
    frames before this one's backward."""
    global _RenderDepth
    if _RenderDepth is None:
        _RenderDepth = _make_function()
    return _RenderDepth.apply(v, sigma, renderer, cam, bool(snapshot), *extra_values)
