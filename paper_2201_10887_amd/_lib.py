"""ctypes view of libhfr's C ABI (``include/hfr.h``): structures, signatures, loading.

Loading imports torch first so that the process holds a single HIP runtime
(torch's); the library then resolves ``libamdhip64.so.7`` to it.  A missing
library is an error: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhfr.so")

HFR_MAX_POLY = 32
HFR_MAX_CASCADES = 8
HFR_MAX_TEX_N = 8192

STATUS = {0: "HFR_OK", -1: "HFR_EINVAL", -2: "HFR_ENOMEM", -3: "HFR_EDEVICE", -4: "HFR_ECAPACITY",
          -5: "HFR_EUNSUPPORTED"}


class HfrError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn}: {STATUS.get(code, code)}: {msg}")
        self.code = code


class Camera(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("yaw", ctypes.c_double), ("pitch", ctypes.c_double),
                ("vfov", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("znear", ctypes.c_double)]


class Domain(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y1", ctypes.c_double), ("zmin", ctypes.c_double), ("zmax", ctypes.c_double)]


class Cascade(ctypes.Structure):
    _fields_ = [("near_d", ctypes.c_double), ("far_d", ctypes.c_double), ("split_d", ctypes.c_double),
                ("origin", ctypes.c_double * 2), ("vhat", ctypes.c_double * 2),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("n", ctypes.c_int32), ("n_poly", ctypes.c_int32), ("poly", (ctypes.c_double * 2) * HFR_MAX_POLY)]


class Leaves(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("packed", ctypes.c_void_p),
                ("level_radius", ctypes.c_void_p), ("rank", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("max_depth", ctypes.c_int32),
                ("cutoff", ctypes.c_float), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("side", ctypes.c_double), ("basis", ctypes.c_int32), ("status", ctypes.c_void_p)]


class BatchField(ctypes.Structure):
    _fields_ = [("leaves", Leaves), ("dom", Domain), ("grad_v", ctypes.c_void_p), ("grad_sigma", ctypes.c_void_p)]


class BatchView(ctypes.Structure):
    _fields_ = [("field", ctypes.c_int32), ("K", ctypes.c_int32), ("N", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("split_lambda", ctypes.c_double), ("overlap", ctypes.c_double), ("c_min", ctypes.c_double),
                ("tex", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("mip", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("hit", ctypes.c_void_p), ("grad_depth", ctypes.c_void_p),
                ("grad_tex", ctypes.c_void_p)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("disc_blocks_per_cu", ctypes.c_int32), ("ray_blocks_per_cu", ctypes.c_int32),
                ("ray_tile_w", ctypes.c_int32), ("disc_grain", ctypes.c_int32), ("ray_queue", ctypes.c_int32),
                ("ray_grain", ctypes.c_int32)]


P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F32 = ctypes.c_float
F64 = ctypes.c_double
PP = ctypes.POINTER

SIGNATURES = {
    "hfr_abi_version": ([], ctypes.c_int),
    "hfr_last_error": ([], ctypes.c_char_p),
    "hfr_runtime_version": ([PP(ctypes.c_int)], I32),
    "hfr_build_quadtree": ([P, I64, F64, F64, F64, I32, F64, PP(P)], I32),
    "hfr_quadtree_size": ([P, PP(I64)], I32),
    "hfr_quadtree_export": ([P, P, P, P, P, P, P, P], I32),
    "hfr_quadtree_destroy": ([P], None),
    "hfr_build_neighbours": ([I64, P, P, P, P, F64, F64, F64, I32, F32, F32, PP(P)], I32),
    "hfr_neighbours_size": ([P, PP(I64)], I32),
    "hfr_neighbours_export": ([P, P, P], I32),
    "hfr_neighbours_destroy": ([P], None),
    "hfr_build_level_index": ([I64, P, P, P, F64, F64, F64, I32, P, P], I32),
    "hfr_fit_cascades": ([PP(Camera), PP(Domain), I32, I32, F64, F64, F64, PP(Cascade)], I32),
    "hfr_fit_cascades_aligned": ([PP(Camera), PP(Domain), I32, I32, F64, F64, F64, PP(Cascade)], I32),
    "hfr_pack_leaves": ([PP(Leaves), P], I32),
    "hfr_discretize": ([PP(Leaves), PP(Domain), PP(Cascade), I32, P, P, P], I32),
    "hfr_discretize_reuse": ([PP(Leaves), PP(Domain), PP(Cascade), I32, PP(Cascade), P, P, P, P, P], I32),
    "hfr_build_maxmip": ([P, I32, I32, P, P], I32),
    "hfr_raycast": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, P, P, P, P], I32),
    "hfr_raycast_backward": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, P, P, P, P], I32),
    "hfr_raycast_split": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, P, P, P, I32, P], I32),
    "hfr_raycast_backward_split": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, P, P, P, I32, P], I32),
    "hfr_quadtree_device_workspace": ([I64, I32, PP(I64)], I32),
    "hfr_neighbours_device_workspace": ([I64, PP(I64)], I32),
    "hfr_build_neighbours_device": ([PP(Leaves), F32, P, P, PP(I64), P], I32),
    "hfr_neighbours_device_fill": ([PP(Leaves), F32, P, P, P], I32),
    "hfr_build_quadtree_device": ([P, I64, F64, F64, F64, I32, F64, P, P, PP(I64), P], I32),
    "hfr_quadtree_device_leaves": ([I64, F64, F64, F64, I32, P, P, I64, P, P, P, P, P, P, P, P], I32),
    "hfr_raycast_static": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, P, P, P], I32),
    "hfr_raycast_static_max_pixels": ([PP(I64)], I32),
    "hfr_raycast_nearer": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, I32, P, P, P, P], I32),
    "hfr_raycast_backward_surface": ([PP(Camera), PP(Domain), PP(Cascade), I32, P, P, I32, P, P, P, P, P], I32),
    "hfr_discretize_backward": ([PP(Leaves), PP(Domain), PP(Cascade), I32, P, P, P, P, P], I32),
    "hfr_batch_plan_create": ([PP(BatchField), I32, PP(BatchView), I32, PP(P)], I32),
    "hfr_batch_plan_destroy": ([P], None),
    "hfr_batch_set_tuning": ([P, PP(BatchTuning)], I32),
    "hfr_batch_long_rays": ([P, P], I32),
    "hfr_batch_set_cameras": ([P, PP(Camera), P], I32),
    "hfr_batch_cascades": ([P, I32, PP(Cascade)], I32),
    "hfr_batch_launch": ([P, P], I32),
    "hfr_batch_launch_backward": ([P, P], I32),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libhfr.so (built by ``paper_2201_10887_amd.build``); raises if it is missing."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  -- one HIP runtime per process: torch's
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2201_10887_amd/build.py (or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def call(name: str, *args) -> int:
    lib = load()
    rc = getattr(lib, name)(*args)
    if rc != 0:
        raise HfrError(name, rc, lib.hfr_last_error().decode())
    return rc
