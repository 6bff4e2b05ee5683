"""Several heightfields in one frame: the nearest surface wins (test infrastructure only).

Section 2 gives the method's input as a terrain model and relative water
depths on the same adaptive grid, and Table 1 times one approximation pass
per heightfield and the ray casting of all of them.  The paper does not
state how the heightfields are combined on screen; this oracle takes the
plain reading that a pixel shows the nearest of the surfaces' first hits
(the earlier surface on a tie), each surface ray cast on its own exactly as
``raycast.raycast`` does.

Pinned by ``tests/test_oracle_composite.py``: two planes, whose depths have
closed forms, give the closed-form nearer depth; a surface composited with
itself changes nothing; a surface lifted above another everywhere wins
everywhere.
"""
from __future__ import annotations

import numpy as np

SURFACE_SHIFT = 29  # the surface index in a hit word sits above the cascade, row and column fields


def nearest(results: list) -> dict:
    """Composite of per-surface ray casts (dicts with ``depth`` and ``hit`` over the same pixels).

    Returns ``depth``, ``surface`` (index of the surface seen, -1 on a miss)
    and ``hit`` (the surface's hit word with the surface index in bits 29-30,
    -1 on a miss)."""
    n = len(results[0]["depth"])
    depth = np.full(n, np.inf)
    surface = np.full(n, -1, np.int64)
    hit = np.full(n, -1, np.int64)
    for s, r in enumerate(results):
        d = np.asarray(r["depth"], np.float64)
        nearer = d < depth
        depth[nearer] = d[nearer]
        surface[nearer] = s
        hit[nearer] = np.asarray(r["hit"], np.int64)[nearer] | (s << SURFACE_SHIFT)
    return {"depth": depth, "surface": surface, "hit": hit}
