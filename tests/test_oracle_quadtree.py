"""Pins of the oracle quadtree against brute-force recomputation from raster blocks."""
import numpy as np
import pytest

from oracle import quadtree
from paper_2201_10887_amd import synth


def _block_mean(dem, level, i, j):
    n = dem.shape[0]
    s = n >> level
    return float(np.mean(dem[j * s:(j + 1) * s, i * s:(i + 1) * s].astype(np.float64)))


def _criterion_bruteforce(dem, level, i, j):
    """Max |second difference| of the four children, recomputed from raster blocks with loops."""
    m = 2 ** (level + 1)

    def mean(a, b):
        a = min(max(a, 0), m - 1)
        b = min(max(b, 0), m - 1)
        return _block_mean(dem, level + 1, a, b)

    best = 0.0
    for cj in (2 * j, 2 * j + 1):
        for ci in (2 * i, 2 * i + 1):
            c = mean(ci, cj)
            best = max(best, abs(mean(ci - 1, cj) + mean(ci + 1, cj) - 2 * c),
                       abs(mean(ci, cj - 1) + mean(ci, cj + 1) - 2 * c))
    return best


def _dfs_order(leafset, depth):
    """Depth-first listing of a leaf set with children (0,0), (1,0), (0,1), (1,1)."""
    out = []

    def rec(l, i, j):
        if (l, i, j) in leafset:
            out.append((l, i, j))
            return
        for dj in (0, 1):
            for di in (0, 1):
                rec(l + 1, 2 * i + di, 2 * j + dj)

    rec(0, 0, 0)
    return out


@pytest.mark.parametrize("seed,tau,depth", [(3, 3.0, 4), (4, 8.0, 5), (5, 1.0, 3), (6, 1e9, 5), (7, 0.0, 4)])
def test_quadtree_against_blocks(seed, tau, depth):
    dem = synth.fbm_dem(32, 5, 0.8, seed, zrange=100.0)
    side = 320.0
    L = quadtree.build_quadtree(dem, side, depth, tau)
    # leaves tile the domain exactly once
    cover = np.zeros((2 ** depth, 2 ** depth), dtype=np.int32)
    for l, i, j in zip(L["level"], L["i"], L["j"]):
        s = 2 ** (depth - l)
        cover[j * s:(j + 1) * s, i * s:(i + 1) * s] += 1
    assert np.all(cover == 1)
    assert np.isclose(np.sum(L["c"].astype(np.float64) ** 2), side * side)
    # geometry and values
    for x, y, c, v, l, i, j in zip(L["x"], L["y"], L["c"], L["v"], L["level"], L["i"], L["j"]):
        assert c == np.float32(side / 2 ** l)
        assert x == np.float32((i + 0.5) * side / 2 ** l) and y == np.float32((j + 0.5) * side / 2 ** l)
        assert abs(float(v) - _block_mean(dem, l, i, j)) <= 1e-4 * max(1.0, abs(float(v)))
    # split rule: leaves above max depth did not qualify, every internal node did
    leafset = set(zip(L["level"].tolist(), L["i"].tolist(), L["j"].tolist()))
    for l, i, j in leafset:
        if l < depth:
            assert _criterion_bruteforce(dem, l, i, j) <= tau + 1e-9
    internal = set()
    for l, i, j in leafset:
        while l > 0:
            l, i, j = l - 1, i // 2, j // 2
            internal.add((l, i, j))
    for l, i, j in internal:
        assert _criterion_bruteforce(dem, l, i, j) > tau - 1e-9
    # depth-first order
    assert list(zip(L["level"].tolist(), L["i"].tolist(), L["j"].tolist())) == _dfs_order(leafset, depth)


def test_extremes():
    dem = synth.fbm_dem(16, 4, 0.8, 9)
    assert len(quadtree.build_quadtree(dem, 16.0, 4, 1e12)["x"]) == 1          # nothing splits
    assert len(quadtree.build_quadtree(dem, 16.0, 4, -1.0)["x"]) == 16 * 16    # everything splits
    flat = np.full((16, 16), 7.0, np.float32)
    L = quadtree.build_quadtree(flat, 16.0, 4, 0.0)
    assert len(L["x"]) == 1 and L["v"][0] == 7.0
    with pytest.raises(ValueError):
        quadtree.build_quadtree(dem, 16.0, 5, 1.0)
