"""Many views of many heightfields per launch (libhfr's ``hfr_batch_*``).

``Field`` is one device-resident heightfield (leaves, level index, per-level
radii, leaf gradients).  ``BatchRenderer`` allocates every view's buffers
once, creates the library plan and runs the batched forward and backward
passes on the current stream; ``capture`` records both into one
``torch.cuda.CUDAGraph`` that stays valid when the cameras change (the
plan keeps every per-camera value in device memory).  Nothing here
computes: all work runs in libhfr.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import api


class Field:
    def __init__(self, leaves: dict, side: float, max_depth: int, cutoff: float, x0: float = 0.0, y0: float = 0.0,
                 device: str = "cuda", with_grads: bool = True, basis="gaussian"):
        import torch
        index = api.build_level_index(leaves, side, max_depth, x0, y0)
        self.L = api.DeviceLeaves(leaves, index, side, max_depth, cutoff, x0, y0, device=device)
        if basis not in ("gaussian", api.BASIS_GAUSSIAN):
            self.L = self.L.with_basis(basis)
        api.pack_leaves(self.L)
        self.dom = _Dom(x0, y0, x0 + side, y0 + side, float(np.min(leaves["v"])), float(np.max(leaves["v"])))
        self.c_min = float(np.min(leaves["c"]))
        self.n = self.L.n
        self.grad_v = torch.zeros(self.n, dtype=torch.float32, device=device) if with_grads else None
        self.grad_sigma = torch.zeros_like(self.grad_v) if with_grads else None

    def refresh(self, stream=None, check: bool = False):
        """Re-derive the packed records after ``L.v`` or ``L.sigma`` changed (``check``: read back the
        leaves' status word, one synchronisation)."""
        api.pack_leaves(self.L, stream, check)


@dataclasses.dataclass
class ViewSpec:
    field: int
    K: int
    N: int
    width: int
    height: int
    split_lambda: float = 0.5
    overlap: float = 0.05


class BatchRenderer:
    def __init__(self, fields: Sequence[Field], views: Sequence[ViewSpec], backward: bool = True,
                 masks: bool = False, tuning: Optional[dict] = None, device: str = "cuda"):
        import torch
        self.fields, self.specs = list(fields), list(views)
        self.bufs = []
        for v in self.specs:
            K, N, W, H = v.K, v.N, v.width, v.height
            b = {
                "tex": torch.empty((K, N, N), dtype=torch.float32, device=device),
                "mip": torch.empty((K, api.mip_size(N)), dtype=torch.float32, device=device),
                "depth": torch.empty((H, W), dtype=torch.float32, device=device),
                "hit": torch.empty((H, W), dtype=torch.int32, device=device),
                "mask": torch.zeros((K, N, (N + 31) // 32), dtype=torch.int32, device=device) if masks else None,
                "grad_depth": torch.zeros((H, W), dtype=torch.float32, device=device) if backward else None,
                "grad_tex": torch.zeros((K, N, N), dtype=torch.float32, device=device) if backward else None,
            }
            self.bufs.append(b)
        fdesc = [{"leaves": f.L, "dom": f.dom, "grad_v": f.grad_v if backward else None,
                  "grad_sigma": f.grad_sigma if backward else None} for f in self.fields]
        vdesc = []
        for v, b in zip(self.specs, self.bufs):
            d = dict(field=v.field, K=v.K, N=v.N, width=v.width, height=v.height, split_lambda=v.split_lambda,
                     overlap=v.overlap, c_min=self.fields[v.field].c_min)
            d.update(b)
            vdesc.append(d)
        self.plan = api.batch_plan_create(fdesc, vdesc)
        self.tuning = dict(disc_blocks_per_cu=4, ray_blocks_per_cu=4, ray_tile_w=32, disc_grain=8, ray_queue=0,
                           ray_grain=8)
        if tuning:
            self.set_tuning(**tuning)

    @property
    def n_views(self) -> int:
        return len(self.specs)

    def set_tuning(self, disc_blocks_per_cu: int = 4, ray_blocks_per_cu: int = 4, ray_tile_w: int = 32,
                   disc_grain: int = 8, ray_queue: int = 0, ray_grain: int = 8):
        api.batch_set_tuning(self.plan, disc_blocks_per_cu, ray_blocks_per_cu, ray_tile_w, disc_grain, ray_queue,
                             ray_grain)
        self.tuning = dict(disc_blocks_per_cu=disc_blocks_per_cu, ray_blocks_per_cu=ray_blocks_per_cu,
                           ray_tile_w=ray_tile_w, disc_grain=disc_grain, ray_queue=ray_queue, ray_grain=ray_grain)

    def set_cameras(self, cams: Sequence, stream=None):
        api.batch_set_cameras(self.plan, cams, stream)

    def cascades(self, view: int):
        return api.batch_cascades(self.plan, view)

    def forward(self, stream=None):
        api.batch_launch(self.plan, stream)

    def backward(self, stream=None):
        api.batch_launch_backward(self.plan, stream)

    def capture(self, backward: bool = True):
        """Record forward (and backward) into a CUDA graph; replay with ``g.replay()`` after
        ``set_cameras`` (on the current stream)."""
        import torch
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up outside the capture
            self.forward(side)
            if backward:
                self.backward(side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s = torch.cuda.current_stream()
            self.forward(s)
            if backward:
                self.backward(s)
        return g


class _Dom:
    def __init__(self, x0, y0, x1, y1, zmin, zmax):
        self.x0, self.y0, self.x1, self.y1, self.zmin, self.zmax = x0, y0, x1, y1, zmin, zmax

    @property
    def extent(self) -> float:
        return max(self.x1 - self.x0, self.y1 - self.y0, self.zmax - self.zmin)
