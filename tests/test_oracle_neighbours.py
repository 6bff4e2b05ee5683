"""Pins of the oracle's per-cell influence lists."""
import math

import numpy as np
import pytest

from oracle import discretize, neighbours
from paper_2201_10887_amd import synth


@pytest.mark.parametrize("seed,depth,p,cutoff", [(1, 5, 0.6, 3.5), (2, 6, 0.45, 3.0), (3, 4, 0.9, 2.0)])
def test_lists_cover_every_influencer(seed, depth, p, cutoff):
    struct = synth.random_leaf_structure(depth, p, seed)
    rng = np.random.default_rng(seed)
    L = synth.leaves_from_structure(struct, 640.0, rng.uniform(0, 200, len(struct)), rng.uniform(0.8, 1.5, len(struct)))
    lists = neighbours.influence_lists(L, cutoff, 1e-3)
    pts = rng.uniform(0, 640.0, (600, 2))
    owner = neighbours.containing_leaf(L, pts[:, 0], pts[:, 1])
    w = discretize.weights(pts, L["x"], L["y"], L["c"], L["sigma"], cutoff)
    allv = (w @ L["v"].astype(np.float64)) / w.sum(axis=1)
    for a in range(len(pts)):
        inf = np.nonzero(w[a] > 0)[0]
        assert np.isin(inf, lists[owner[a]]).all()
        j = lists[owner[a]]
        lv = (w[a, j] @ L["v"][j].astype(np.float64)) / w[a, j].sum()
        assert abs(lv - allv[a]) < 1e-12 * 200
    # the containing cell always influences its own points when cutoff*sigma > sqrt(2)/2
    for a in range(len(pts)):
        assert w[a, owner[a]] > 0 or cutoff * L["sigma"][owner[a]] <= math.sqrt(0.5)
