"""Maximum mipmap over a cascade texture (FP64 test infrastructure).

Section 5 uses the maximum mipmaps of Tevs et al. 2008 for empty-space
skipping without describing them; this follows that public definition:

* Level 0 is indexed by texture cell: ``M0[j, i]`` is the largest of the
  cell's four corner texels when all four are visible, ``-inf`` otherwise;
  the last row and column (no cell) are ``-inf``.  It is ``N x N``.
* ``M_{l+1}[j, i]`` is the largest of the 2x2 block ``M_l[2j:2j+2, 2i:2i+2]``,
  down to a single value: ``log2(N) + 1`` levels.

Pinned by ``tests/test_oracle_maxmip.py``: every node equals the brute-force
maximum over the corner texels of the cells in its footprint.
"""
from __future__ import annotations

import numpy as np


def level0(tex: np.ndarray) -> np.ndarray:
    N = tex.shape[0]
    corners = np.stack([tex[:-1, :-1], tex[:-1, 1:], tex[1:, :-1], tex[1:, 1:]])
    ok = np.all(np.isfinite(corners), axis=0)
    m0 = np.full((N, N), -np.inf)
    m0[:-1, :-1] = np.where(ok, corners.max(axis=0), -np.inf)
    return m0


def maxmip(tex: np.ndarray) -> list:
    """List of levels ``[M0 (N x N), M1 (N/2 x N/2), ..., (1 x 1)]``."""
    levels = [level0(np.asarray(tex, np.float64))]
    while levels[-1].shape[0] > 1:
        m = levels[-1]
        levels.append(np.maximum(np.maximum(m[0::2, 0::2], m[0::2, 1::2]), np.maximum(m[1::2, 0::2], m[1::2, 1::2])))
    return levels


def flatten(levels: list) -> np.ndarray:
    """Levels concatenated finest first, each row-major: ``(4 N^2 - 1) / 3`` values."""
    return np.concatenate([m.ravel() for m in levels])
