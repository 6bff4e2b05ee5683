"""Pinhole camera and per-pixel rays (test infrastructure, FP64).

Section 5 casts one ray per pixel; the paper states no camera model, so this
is a reading: world x east, y north, z up; the forward vector is
``(sin yaw cos pitch, cos yaw cos pitch, sin pitch)`` (yaw 0 looks along +y,
pitch < 0 looks down); right is horizontal, up completes the frame; the
image plane spans ``tan(vfov/2)`` vertically and ``tan(vfov/2) * W / H``
horizontally; pixel ``(col, row)`` is sampled at its centre with row 0 at the
top; rays are unit length so the ray parameter is Euclidean distance.

Pinned by ``tests/test_oracle_cascades.py::test_camera_frame_and_fov``
(orthonormal frame, centre pixel along forward for odd sizes, corner rays on
the frustum edges).
"""
from __future__ import annotations

import math

import numpy as np


def basis(cam) -> tuple:
    """``(forward, right, up)`` unit vectors of the camera frame."""
    cy, sy = math.cos(cam.yaw), math.sin(cam.yaw)
    cp, sp = math.cos(cam.pitch), math.sin(cam.pitch)
    fwd = np.array([sy * cp, cy * cp, sp])
    right = np.array([cy, -sy, 0.0])
    up = np.cross(right, fwd)
    return fwd, right, up


def ray_directions(cam, cols: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Unit directions ``(n, 3)`` of the rays through pixel centres ``(cols, rows)``."""
    fwd, right, up = basis(cam)
    ty = math.tan(0.5 * cam.vfov)
    tx = ty * cam.width / cam.height
    sx = (np.asarray(cols, np.float64) + 0.5) / cam.width * 2.0 - 1.0
    sy = 1.0 - (np.asarray(rows, np.float64) + 0.5) / cam.height * 2.0
    d = fwd[None, :] + (sx * tx)[:, None] * right[None, :] + (sy * ty)[:, None] * up[None, :]
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def all_pixels(cam) -> tuple:
    """Column and row index of every pixel, row-major."""
    rows, cols = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return cols.ravel(), rows.ravel()
