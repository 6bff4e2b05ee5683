"""Adaptive quadtree over a square raster (test infrastructure, FP64).

The paper takes the adaptive grid from the flood simulation (Section 2: a
digital elevation model and water depths defined at the cell centres of an
adaptive grid; Table 1 lists cell sizes from 0.75 m to 96 m).  It never says
how such a grid is refined, so the rule here is a reading:

* ``M[l]`` is the mean raster at level ``l`` (``2**l`` nodes per side), built
  from the raster by averaging 2x2 blocks in the fixed order
  ``((a + b) + (c + d)) * 0.25`` with ``a, b`` the lower pair along x.
* A node ``(l, i, j)`` with ``l < max_depth`` splits when the largest absolute
  second difference (along x or y, edge samples replicated) of the level
  ``l + 1`` means under it exceeds ``tau``.  The level-``l`` version of the
  same test is identically zero at the root, hence the children.
* A leaf's value is its mean ``M[l][j, i]``; its centre is the node centre.
* Leaves are listed in depth-first order with children in the order
  ``(2i, 2j), (2i+1, 2j), (2i, 2j+1), (2i+1, 2j+1)`` (Morton order).

Pinned by ``tests/test_oracle_quadtree.py``: leaves tile the domain, each leaf
value equals the brute-force mean of its raster block, and the split rule
recomputed from raster blocks holds at every leaf and every internal node.
"""
from __future__ import annotations

import numpy as np


def mean_pyramid(dem: np.ndarray) -> list:
    """``M[l]`` for ``l = 0 .. log2(n)``, FP64, with ``M[log2 n]`` the raster itself."""
    levels = [np.asarray(dem, dtype=np.float64)]
    while levels[-1].shape[0] > 1:
        m = levels[-1]
        levels.append(((m[0::2, 0::2] + m[0::2, 1::2]) + (m[1::2, 0::2] + m[1::2, 1::2])) * 0.25)
    return levels[::-1]


def second_difference(m: np.ndarray) -> np.ndarray:
    """``max(|d2x|, |d2y|)`` per sample with replicated edges, ``d2x = (left + right) - 2 centre``."""
    left = np.concatenate([m[:, :1], m[:, :-1]], axis=1)
    right = np.concatenate([m[:, 1:], m[:, -1:]], axis=1)
    down = np.concatenate([m[:1, :], m[:-1, :]], axis=0)
    up = np.concatenate([m[1:, :], m[-1:, :]], axis=0)
    d2x = (left + right) - 2.0 * m
    d2y = (down + up) - 2.0 * m
    return np.maximum(np.abs(d2x), np.abs(d2y))


def split_criterion(M: list, level: int) -> np.ndarray:
    """Criterion of every node at ``level``: max second difference of its four children."""
    s = second_difference(M[level + 1])
    return np.maximum(np.maximum(s[0::2, 0::2], s[0::2, 1::2]), np.maximum(s[1::2, 0::2], s[1::2, 1::2]))


def morton_key(level: np.ndarray, i: np.ndarray, j: np.ndarray, depth: int) -> np.ndarray:
    """Z-order key of each node's lower-left finest cell (x bit below y bit)."""
    shift = (depth - level).astype(np.uint64)
    x = i.astype(np.uint64) << shift
    y = j.astype(np.uint64) << shift
    key = np.zeros_like(x)
    for b in range(depth):
        key |= ((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((y >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def build_quadtree(dem: np.ndarray, side: float, max_depth: int, tau: float,
                   x0: float = 0.0, y0: float = 0.0) -> dict:
    """Leaves of the adaptive quadtree over ``dem`` (square, power-of-two side).

    Returns float32 ``x, y, c, v`` (centre, size, mean value) and int32
    ``level, i, j`` in depth-first (Morton) order.
    """
    n = dem.shape[0]
    depth_raster = int(round(np.log2(n)))
    if dem.shape != (n, n) or 2 ** depth_raster != n:
        raise ValueError("raster must be square with a power-of-two side")
    if not 0 <= max_depth <= depth_raster:
        raise ValueError("max_depth must lie in [0, log2(raster side)]")
    M = mean_pyramid(dem)
    lv, li, lj = [], [], []
    nodes = np.zeros((1, 2), dtype=np.int64)  # (i, j) of live nodes at this level
    for level in range(max_depth + 1):
        if level < max_depth:
            crit = split_criterion(M, level)
            split = crit[nodes[:, 1], nodes[:, 0]] > tau
        else:
            split = np.zeros(len(nodes), dtype=bool)
        keep = nodes[~split]
        lv.append(np.full(len(keep), level, dtype=np.int64))
        li.append(keep[:, 0])
        lj.append(keep[:, 1])
        parents = nodes[split]
        kids = []
        for dj in (0, 1):
            for di in (0, 1):
                kids.append(np.stack([2 * parents[:, 0] + di, 2 * parents[:, 1] + dj], axis=1))
        nodes = np.concatenate(kids, axis=0) if len(parents) else np.zeros((0, 2), dtype=np.int64)
    level = np.concatenate(lv)
    i = np.concatenate(li)
    j = np.concatenate(lj)
    order = np.argsort(morton_key(level, i, j, max_depth), kind="stable")
    level, i, j = level[order], i[order], j[order]
    c = side / 2.0 ** level
    v = np.array([M[l][jj, ii] for l, ii, jj in zip(level, i, j)]) if len(level) < 4096 else \
        _gather_values(M, level, i, j)
    return dict(x=(x0 + (i + 0.5) * c).astype(np.float32), y=(y0 + (j + 0.5) * c).astype(np.float32),
                c=c.astype(np.float32), v=v.astype(np.float32),
                level=level.astype(np.int32), i=i.astype(np.int32), j=j.astype(np.int32))


def _gather_values(M, level, i, j):
    v = np.empty(len(level), dtype=np.float64)
    for l in np.unique(level):
        sel = level == l
        v[sel] = M[l][j[sel], i[sel]]
    return v
