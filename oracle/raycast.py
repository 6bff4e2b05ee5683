"""FP64 ray casting over cascade textures (Section 5): Python side of ``oracle/c``.

The cell walk, the patch root and the overlap blend are described in the
header of ``oracle/c/raycast_oracle.c``.  This module builds the rays
(``oracle.camera``), packs the cascades and reads the results back.

Pinned by ``tests/test_oracle_raycast.py``: a tilted plane (bilinear
interpolation is exact, so the depth has a closed form), a constant field,
testing every cell of the texture by brute force, dense marching with
bisection, and the overlap blend against closed forms on cascades of
different constant heights (both sweep directions, at the overlap's ends and
at weights strictly inside).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from .camera import all_pixels, ray_directions

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.library_path("raycast_oracle")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SOURCES["raycast_oracle"]):
            _build.build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_raycast.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_raycast.restype = ctypes.c_int
        lib.oracle_cell_root.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, P]
        lib.oracle_cell_root.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def cascade_params(cascades) -> np.ndarray:
    rows = []
    for c in cascades:
        rows.append([c.near, c.far, c.split, c.origin[0], c.origin[1], c.vhat[0], c.vhat[1],
                     c.x0, c.y0, c.hx, c.hy, float(c.n)])
    return np.ascontiguousarray(np.array(rows, np.float64))


def cast_rays(origins: np.ndarray, dirs: np.ndarray, dom, cascades, tex: np.ndarray, threads: int = 1) -> dict:
    """Cast arbitrary rays; ``tex`` is ``[K][N][N]`` heights (read as FP64), ``-inf`` = invisible."""
    lib = _load()
    n = len(dirs)
    o = np.ascontiguousarray(np.broadcast_to(np.asarray(origins, np.float64), (n, 3)))
    d = np.ascontiguousarray(dirs, np.float64)
    domv = np.array([dom.x0, dom.y0, dom.x1, dom.y1, dom.zmin, dom.zmax], np.float64)
    cas = cascade_params(cascades)
    t = np.ascontiguousarray(tex, np.float64)
    if t.shape != (len(cascades), cascades[0].n, cascades[0].n):
        raise ValueError("texture stack shape does not match the cascades")
    out = dict(depth=np.empty(n), hit=np.empty(n, np.int32), rec=np.empty((n, 8), np.int32),
               val=np.empty((n, 8)), coef=np.empty((n, 2)))
    rc = lib.oracle_raycast(n, _ptr(o), _ptr(d), _ptr(domv), len(cascades), _ptr(cas), _ptr(t),
                            _ptr(out["depth"]), _ptr(out["hit"]), _ptr(out["rec"]), _ptr(out["val"]),
                            _ptr(out["coef"]), int(threads))
    if rc != 0:
        raise ValueError("oracle_raycast rejected its arguments")
    out["dirs"] = d
    return out


def raycast(cam, dom, cascades, tex: np.ndarray, cols=None, rows=None, threads: int = 1) -> dict:
    """Depth and hit id for pixels ``(cols, rows)`` (all pixels when omitted)."""
    if cols is None:
        cols, rows = all_pixels(cam)
    dirs = ray_directions(cam, cols, rows)
    out = cast_rays(np.asarray(cam.pos, np.float64), dirs, dom, cascades, tex, threads)
    out["cols"], out["rows"] = np.asarray(cols), np.asarray(rows)
    return out


def cell_root(origin, direction, cas, tex_k: np.ndarray, i: int, j: int):
    """First root of one ray inside cell ``(i, j)`` (whole piece in the cell), or ``None``."""
    lib = _load()
    o = np.ascontiguousarray(origin, np.float64)
    d = np.ascontiguousarray(direction, np.float64)
    p = cascade_params([cas])[0].copy()
    t = np.ascontiguousarray(tex_k, np.float64)
    res = np.zeros(1)
    ok = lib.oracle_cell_root(_ptr(o), _ptr(d), _ptr(p), _ptr(t), int(i), int(j), _ptr(res))
    return float(res[0]) if ok else None


def unpack_hit(h: np.ndarray) -> tuple:
    h = np.asarray(h, np.int64)
    return (h >> 26) & 31, (h >> 13) & 8191, h & 8191
