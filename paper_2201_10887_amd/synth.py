"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds none of the renderer's arithmetic: it only draws terrain
rasters, camera poses and small hand-made test fields.  The paper measures on
four real flood-simulation scenarios (Section 6, Table 1) whose elevation
models are not available; fractal (fBm) terrain of the same size range stands
in for them.

Terrain recipe: value noise on an integer lattice, octave ``o`` (1-based) has
``2**o`` lattice cells across the domain and amplitude ``2**(-hurst*o)``; the
lattice values are uniform in [-1, 1] from ``numpy.random.default_rng(seed)``;
the interpolation is separable with the quintic fade; heights are min-max
rescaled to ``[0, zrange]``.  Optional ridged mountains add
``mountain_height * mask * (1 - |noise|)**2`` where ``mask`` is a smooth blob
field from the same generator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np


def _fade(f: np.ndarray) -> np.ndarray:
    return f * f * f * (f * (f * 6.0 - 15.0) + 10.0)


def _lattice(cells: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((cells + 1, cells + 1)) * 2.0 - 1.0


def _interp_weights(n: int, cells: int):
    s = (np.arange(n, dtype=np.float64) + 0.5) / n * cells
    i = np.minimum(np.floor(s).astype(np.int64), cells - 1)
    return i, _fade(s - i)


def _value_noise(n: int, cells: int, rng: np.random.Generator, dtype=np.float64, xp=None) -> np.ndarray:
    """One octave of value noise sampled at the centres of an ``n x n`` raster.

    ``xp`` (a torch device) runs the separable interpolation in torch there;
    the lattice values come from ``rng`` either way."""
    g = _lattice(cells, rng)
    i, f = _interp_weights(n, cells)
    if xp is not None:
        import torch
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        g = torch.as_tensor(g, device=xp).to(tdt)
        i = torch.as_tensor(i, device=xp)
        f = torch.as_tensor(f, device=xp).to(tdt)
        rows = g[i] * (1.0 - f)[:, None] + g[i + 1] * f[:, None]
        return rows[:, i] * (1.0 - f)[None, :] + rows[:, i + 1] * f[None, :]
    g = g.astype(dtype)
    f = f.astype(dtype)
    rows = g[i] * (1.0 - f)[:, None] + g[i + 1] * f[:, None]
    return rows[:, i] * (1.0 - f)[None, :] + rows[:, i + 1] * f[None, :]


def fbm_dem(n: int, octaves: int, hurst: float, seed: int, zrange: float = 300.0,
            mountains: float = 0.0, device=None) -> np.ndarray:
    """Seeded fBm raster, ``float32[n][n]`` (row = y index, column = x index).

    ``device`` (e.g. "cuda") runs the interpolation in torch on that device
    (the same lattice values and formula; FP32 rounding order may differ):
    minutes of NumPy work at 16384^2 become seconds."""
    if n <= 0 or n & (n - 1):
        raise ValueError("raster side must be a power of two")
    rng = np.random.default_rng(seed)
    dtype = np.float64 if n <= 4096 else np.float32
    if device is not None:
        import torch
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        zeros = lambda: torch.zeros((n, n), dtype=tdt, device=device)
        vmax = lambda a: float(a.max())
        vmin = lambda a: float(a.min())
        absf = torch.abs
        clip = lambda a, lo, hi: torch.clamp(a, lo, hi)
        xp = device
    else:
        zeros = lambda: np.zeros((n, n), dtype=dtype)
        vmax = lambda a: float(a.max())
        vmin = lambda a: float(a.min())
        absf = np.abs
        clip = np.clip
        xp = None
    acc = zeros()
    for o in range(1, octaves + 1):
        acc += _value_noise(n, 2 ** o, rng, dtype, xp) * float(dtype(2.0 ** (-hurst * o)))
    lo, hi = vmin(acc), vmax(acc)
    acc = (acc - lo) * float(dtype(zrange / max(hi - lo, 1e-30)))
    if mountains > 0.0:
        mask = _value_noise(n, 4, rng, dtype, xp)
        mask = clip(mask * 1.5, 0.0, 1.0)
        ridge = zeros()
        for o in range(3, min(octaves, 11) + 1):
            ridge += (1.0 - absf(_value_noise(n, 2 ** o, rng, dtype, xp))) ** 2 * float(dtype(2.0 ** (-hurst * (o - 3))))
        ridge /= max(vmax(ridge), 1e-30)
        acc += float(dtype(mountains)) * mask * ridge
    if device is not None:
        return acc.float().cpu().numpy()
    return acc.astype(np.float32)


def water_surface(leaves: dict, side: float, seed: int, wet_fraction: float = 0.3, relief: float = 4.0,
                  dry_drop: float = 1.0, raster_n: int = 512, x0: float = 0.0, y0: float = 0.0) -> np.ndarray:
    """Per-leaf value of a synthetic water surface on the terrain's own cells, ``float32[n]``.

    Stands in for the relative water depths of a flood simulation on the same
    adaptive grid: a seeded smooth flood level (four octaves of the fBm
    generator on a ``raster_n^2`` lattice, ``relief`` metres of variation,
    sampled bilinearly at the cell centres) is raised until about
    ``wet_fraction`` of the cells lie below it.  A wet cell holds terrain
    value plus relative depth (the level there); a dry cell holds its terrain
    value minus ``dry_drop``, so that the terrain is the nearer surface."""
    lvl = fbm_dem(raster_n, 4, 0.8, seed, zrange=relief).astype(np.float64)
    gx = np.clip((np.asarray(leaves["x"], np.float64) - x0) / side * raster_n - 0.5, 0.0, raster_n - 1.0)
    gy = np.clip((np.asarray(leaves["y"], np.float64) - y0) / side * raster_n - 0.5, 0.0, raster_n - 1.0)
    i0 = np.minimum(gx.astype(np.int64), raster_n - 2)
    j0 = np.minimum(gy.astype(np.int64), raster_n - 2)
    fx, fy = gx - i0, gy - j0
    level = ((lvl[j0, i0] * (1 - fx) + lvl[j0, i0 + 1] * fx) * (1 - fy)
             + (lvl[j0 + 1, i0] * (1 - fx) + lvl[j0 + 1, i0 + 1] * fx) * fy)
    v = np.asarray(leaves["v"], np.float64)
    level += np.quantile(v - level, wet_fraction)
    depth = level - v
    return np.where(depth > 0.0, v + depth, v - dry_drop).astype(np.float32)


@dataclasses.dataclass(frozen=True)
class Camera:
    """Pinhole camera: world x east, y north, z up; yaw 0 looks along +y, pitch < 0 looks down."""
    pos: Tuple[float, float, float]
    yaw: float
    pitch: float
    vfov: float
    width: int
    height: int
    znear: float = 1.0


@dataclasses.dataclass(frozen=True)
class Domain:
    x0: float
    y0: float
    x1: float
    y1: float
    zmin: float
    zmax: float

    @property
    def extent(self) -> float:
        return max(self.x1 - self.x0, self.y1 - self.y0, self.zmax - self.zmin)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic scene: terrain raster, quadtree parameters, RBF shape, camera, cascades."""
    name: str
    side: float            # domain side (m); the domain is [0, side]^2
    dem_n: int             # raster samples per side (power of two)
    octaves: int
    hurst: float
    seed: int
    max_depth: int         # quadtree depth; finest cell = side / 2**max_depth
    tau: float             # refinement threshold (m)
    sigma: float           # Gaussian width in units of the cell size
    cutoff: float          # truncation radius in units of sigma
    cam_xy: Tuple[float, float]  # camera position as a fraction of the side
    cam_alt: float         # camera height above the terrain sample under it (m)
    yaw_deg: float
    pitch_deg: float
    vfov_deg: float
    width: int
    height: int
    cascades: int          # K
    tex_n: int             # N texels per cascade side
    split_lambda: float    # blend of logarithmic (1) and uniform (0) splits
    overlap: float = 0.05  # overlap width as a fraction of the cascade depth range
    mountains: float = 0.0
    zrange: float = 300.0
    water_seed: int = 0    # > 0: a second surface, water on the terrain's cells (water_surface)
    water_wet: float = 0.3

    @property
    def c_min(self) -> float:
        return self.side / 2 ** self.max_depth

    @property
    def spacing(self) -> float:
        return self.side / self.dem_n


# The quadtree thresholds tau were bisected once against the stated leaf
# counts (~2k for the tiny scene, ~4M for the medium one): with the
# second-difference rule the stated 0.5 m and 0.2 m refine every node to the
# maximum depth (4096 and 16.7M leaves).
TINY = Workload(name="tiny: 1 km fBm, 2048 leaves (depth 6), 2x256^2 cascades, 256x256",
              side=1024.0, dem_n=256, octaves=8, hurst=0.8, seed=0, max_depth=6, tau=11.25,
              sigma=1.5, cutoff=3.0, cam_xy=(0.5, 0.05), cam_alt=100.0, yaw_deg=0.0,
              pitch_deg=-20.0, vfov_deg=60.0, width=256, height=256, cascades=2, tex_n=256,
              split_lambda=1.0)

MEDIUM = Workload(name="medium: 40.96 km fBm, 3.97M leaves (depth 12), 4x2048^2 cascades, 1920x1080",
              side=40960.0, dem_n=4096, octaves=12, hurst=0.8, seed=1, max_depth=12, tau=0.68,
              sigma=1.0, cutoff=3.5, cam_xy=(0.5, 0.05), cam_alt=200.0, yaw_deg=0.0,
              pitch_deg=-10.0, vfov_deg=60.0, width=1920, height=1080, cascades=4, tex_n=2048,
              split_lambda=0.5)

# Paper-shaped context: the medium terrain with three 1024^2 cascades,
# logarithmic splits, sigma 1 and a 3.5 sigma cutoff at 1080p (Section 6).
PAPER = dataclasses.replace(MEDIUM, name="paper-shaped: medium terrain, 3x1024^2 cascades, 1920x1080",
                         cascades=3, tex_n=1024, split_lambda=1.0)

# Large: 163.84 km at 10 m finest cells (depth 14) with ridged mountains up to
# 1.5 km over the 300 m fBm; tau bisected once to the stated ~64M leaves
# (64,092,346); a grazing 3 degree view at 3840 x 2160 with 4 x 4096^2 cascades.
LARGE = Workload(name="large: 163.84 km fBm + ridged mountains, 64.1M leaves (depth 14), 4x4096^2 cascades, 3840x2160",
              side=163840.0, dem_n=16384, octaves=14, hurst=0.8, seed=2, max_depth=14, tau=0.9728,
              sigma=1.0, cutoff=3.5, cam_xy=(0.5, 0.05), cam_alt=200.0, yaw_deg=0.0,
              pitch_deg=-3.0, vfov_deg=60.0, width=3840, height=2160, cascades=4, tex_n=4096,
              split_lambda=0.5, mountains=1500.0)

MEDIUM_WATER = dataclasses.replace(
    MEDIUM, name="medium + water: the 40.96 km scene with a flood surface on 30 % of its cells (two surfaces), "
                 "4x2048^2 cascades each, 1920x1080", water_seed=91)

WORKLOADS = {"tiny": TINY, "medium": MEDIUM, "paper": PAPER, "large": LARGE, "medium_water": MEDIUM_WATER}


def domain_of(w: Workload, dem: np.ndarray) -> Domain:
    return Domain(0.0, 0.0, w.side, w.side, float(dem.min()), float(dem.max()))


def camera_of(w: Workload, dem: np.ndarray, width: Optional[int] = None,
              height: Optional[int] = None) -> Camera:
    """Camera pose of a workload: position from the raster sample under it plus altitude."""
    n = dem.shape[0]
    cx, cy = w.cam_xy[0] * w.side, w.cam_xy[1] * w.side
    ix = min(int(cx / w.spacing), n - 1)
    iy = min(int(cy / w.spacing), n - 1)
    z = float(dem[iy, ix]) + w.cam_alt
    return Camera(pos=(cx, cy, z), yaw=math.radians(w.yaw_deg), pitch=math.radians(w.pitch_deg),
                  vfov=math.radians(w.vfov_deg), width=width or w.width, height=height or w.height)


def camera_path(cam: Camera, frames: int, step: float, yaw_step_deg: float = 0.0,
                climb: float = 0.0) -> List[Camera]:
    """A flight: ``frames`` poses starting at ``cam``, each ``step`` metres further along the horizontal
    view direction (and ``climb`` metres up), turning by ``yaw_step_deg`` per frame."""
    out = []
    x, y, z = cam.pos
    yaw = cam.yaw
    for _ in range(frames):
        out.append(Camera(pos=(x, y, z), yaw=yaw, pitch=cam.pitch, vfov=cam.vfov, width=cam.width,
                          height=cam.height))
        x += step * math.sin(yaw)
        y += step * math.cos(yaw)
        z += climb
        yaw += math.radians(yaw_step_deg)
    return out


def random_cameras(dem: np.ndarray, side: float, count: int, seed: int,
                   sizes: List[Tuple[int, int]]) -> List[Camera]:
    """Random poses above the terrain: xy in the inner 80 %, 50-500 m up, pitch -30..-3 deg."""
    rng = np.random.default_rng(seed)
    n = dem.shape[0]
    out = []
    for _ in range(count):
        cx, cy = rng.uniform(0.1, 0.9, size=2) * side
        ix = min(int(cx / side * n), n - 1)
        iy = min(int(cy / side * n), n - 1)
        z = float(dem[iy, ix]) + rng.uniform(50.0, 500.0)
        w, h = sizes[rng.integers(len(sizes))]
        out.append(Camera(pos=(cx, cy, z), yaw=rng.uniform(0, 2 * math.pi),
                          pitch=math.radians(rng.uniform(-30.0, -3.0)), vfov=math.radians(60.0),
                          width=int(w), height=int(h)))
    return out


def random_leaf_structure(depth: int, p_split: float, seed: int) -> List[Tuple[int, int, int]]:
    """Random quadtree leaf set ``[(level, i, j)]`` (no values): each node splits with ``p_split``."""
    rng = np.random.default_rng(seed)
    leaves = []
    stack = [(0, 0, 0)]
    while stack:
        l, i, j = stack.pop()
        if l < depth and (l == 0 or rng.random() < p_split):
            for dj in (1, 0):
                for di in (1, 0):
                    stack.append((l + 1, 2 * i + di, 2 * j + dj))
        else:
            leaves.append((l, i, j))
    return leaves


def leaves_from_structure(struct: List[Tuple[int, int, int]], side: float, values: np.ndarray,
                          sigma: np.ndarray) -> dict:
    """Float32 leaf arrays (centre, size, value, sigma) for a leaf structure on ``[0, side]^2``."""
    lv = np.array([s[0] for s in struct], dtype=np.int32)
    ii = np.array([s[1] for s in struct], dtype=np.float64)
    jj = np.array([s[2] for s in struct], dtype=np.float64)
    c = side / 2.0 ** lv
    return dict(x=((ii + 0.5) * c).astype(np.float32), y=((jj + 0.5) * c).astype(np.float32),
                c=c.astype(np.float32), v=np.asarray(values, np.float32),
                sigma=np.asarray(sigma, np.float32), level=lv)


def resample_raster(dem: np.ndarray, side: float, x0: float, y0: float, hx: float, hy: float, n: int) -> np.ndarray:
    """Nearest raster sample at each point ``(x0 + i hx, y0 + j hy)``: a stand-in texture of a given shape."""
    m = dem.shape[0]
    gx = np.clip(np.floor((x0 + np.arange(n) * hx) / side * m).astype(np.int64), 0, m - 1)
    gy = np.clip(np.floor((y0 + np.arange(n) * hy) / side * m).astype(np.int64), 0, m - 1)
    return dem[np.ix_(gy, gx)].astype(np.float32)


# ------------------------------------------------------------------ batched workload
#
# Many views of several heightfields of uneven size: 8 fields whose leaf
# counts are drawn log-uniformly between 10k and 4M (depth 8 to 12, finest
# cell 10 m, side 10 m * 2^depth), and 64 cameras, camera c viewing field
# c mod 8 with a resolution drawn from {256^2, 512^2, 1280x720, 1920x1080},
# K drawn from {2, 3, 4}, and a pose as ``random_cameras`` draws it.

BATCH_RESOLUTIONS = [(256, 256), (512, 512), (1280, 720), (1920, 1080)]


@dataclasses.dataclass(frozen=True)
class BatchFieldSpec:
    depth: int
    side: float
    dem_n: int
    octaves: int
    seed: int
    target_leaves: int


@dataclasses.dataclass(frozen=True)
class BatchViewSpec:
    field: int
    width: int
    height: int
    K: int


# Refinement thresholds of the eight batch fields (seed 1004): bisected once, on a log scale, until the
# quadtree's leaf count came within 15 % of each field's drawn target (9055, 19666, 21883, 105007, 437497,
# 1639447, 23554 and 272578 leaves).
BATCH_TAU = (6.97831, 6.97831, 5.62341, 2.37137, 1.71544, 0.897687, 5.04807, 2.12875)


def batch_fields(n_fields: int = 8, seed: int = 1004, lo: float = 1e4, hi: float = 4e6) -> List[BatchFieldSpec]:
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n_fields):
        target = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        depth = int(min(12, max(8, math.ceil(math.log(target, 4)) + 1)))
        n = 2 ** depth
        out.append(BatchFieldSpec(depth=depth, side=10.0 * n, dem_n=n, octaves=depth, seed=seed + 1 + f,
                                  target_leaves=target))
    return out


def batch_views(n_views: int = 64, n_fields: int = 8, seed: int = 1004) -> List[BatchViewSpec]:
    rng = np.random.default_rng(seed + 100)
    out = []
    for c in range(n_views):
        w, h = BATCH_RESOLUTIONS[rng.integers(len(BATCH_RESOLUTIONS))]
        out.append(BatchViewSpec(field=c % n_fields, width=w, height=h, K=int(rng.integers(2, 5))))
    return out


def batch_cameras(dems: List[np.ndarray], fields: List[BatchFieldSpec], views: List[BatchViewSpec],
                  seed: int = 1004) -> List[Camera]:
    out = []
    for c, v in enumerate(views):
        f = fields[v.field]
        out.append(random_cameras(dems[v.field], f.side, 1, seed + 1000 + c, [(v.width, v.height)])[0])
    return out
