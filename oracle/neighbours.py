"""Per-cell lists of potentially influencing cells (Section 4), FP64 test infrastructure.

The set of cells influencing a position depends only on the grid, so the
paper precomputes, per cell, a buffer of all cells that may influence any
position inside it.  Reading: the list of cell ``i`` holds every cell ``j``
whose truncation radius ``R_j = cutoff * sigma_j * c_j``, widened by the
relative ``slack``, reaches the closed square of ``i``:
``dist(p_j, square_i)^2 < (R_j (1 + slack))^2``.  Any ``j`` with
``w_j(p) > 0`` for a ``p`` in square ``i`` is then listed, so the list sum
equals the sum over all cells.

Pinned by ``tests/test_oracle_neighbours.py`` (coverage of every influencer
of random points, and equality of list sums with all-leaves sums).
"""
from __future__ import annotations

import numpy as np


def square_distance2(px, py, cx, cy, half):
    """Squared distance of points to axis-aligned squares (centre, half side)."""
    dx = np.maximum(np.abs(px - cx) - half, 0.0)
    dy = np.maximum(np.abs(py - cy) - half, 0.0)
    return dx * dx + dy * dy


def influence_lists(leaves: dict, cutoff: float, slack: float) -> list:
    """Brute force over all pairs; list ``i`` sorted by leaf index."""
    x = np.asarray(leaves["x"], np.float64)
    y = np.asarray(leaves["y"], np.float64)
    c = np.asarray(leaves["c"], np.float64)
    s = np.asarray(leaves["sigma"], np.float64)
    R = ((cutoff * s) * c) * (1.0 + slack)
    out = []
    for i in range(len(x)):
        d2 = square_distance2(x, y, x[i], y[i], 0.5 * c[i])
        out.append(np.nonzero(d2 < R * R)[0])
    return out


def containing_leaf(leaves: dict, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Index of a leaf whose closed square contains each point (brute force)."""
    x = np.asarray(leaves["x"], np.float64)
    y = np.asarray(leaves["y"], np.float64)
    h = 0.5 * np.asarray(leaves["c"], np.float64)
    out = np.empty(len(px), np.int64)
    for a in range(len(px)):
        inside = np.nonzero((np.abs(px[a] - x) <= h) & (np.abs(py[a] - y) <= h))[0]
        out[a] = inside[0]
    return out
