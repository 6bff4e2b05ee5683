"""Texel budget and measured launch-shape tuning for batched rendering.

``texel_budget`` picks each view's cascade resolution N: one texel per pixel
of the image's larger side (the paper pairs 1024^2 cascades with 1080p,
Section 6; a power of two at least as large as the image side keeps the
nearest cascade from being magnified), clamped to [n_min, n_max], then
halved view by view (largest N first) until the batch's sum of K N^2 fits the
budget.  ``tune`` times every launch shape of a grid on the actual batch
(forward, or forward + backward) with HIP events and keeps the fastest; the
choice is cached in a JSON file keyed by the batch's shape and the device,
so a later run with the same shape skips the measurements.  ``tune_budget``
chooses the texel budget itself by measurement: the largest budget of a
ladder whose tuned batch step fits a time target.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "_build", "autotune.json")

DEFAULT_GRID = {
    "disc_blocks_per_cu": (4, 7),
    "disc_grain": (8, 16),
    "ray_blocks_per_cu": (2, 4),
    "ray_tile_w": (16, 32),
    "ray_queue": (0, 1),
    "ray_grain": (4, 8, 16),
}


def _next_pow2(x: int) -> int:
    n = 1
    while n < x:
        n *= 2
    return n


def texel_budget(views: Sequence[Tuple[int, int, int]], budget_texels: int = 1 << 28, n_min: int = 256,
                 n_max: int = 2048) -> List[int]:
    """N per view for ``views`` = [(width, height, K)]."""
    ns = [min(max(_next_pow2(max(w, h)), n_min), n_max) for (w, h, _) in views]
    total = lambda: sum(k * n * n for (_, _, k), n in zip(views, ns))
    while total() > budget_texels:
        big = max(range(len(ns)), key=lambda a: (ns[a], -a))
        if ns[big] <= n_min:
            break
        ns[big] //= 2
    return ns


def signature(renderer, backward: bool) -> str:
    import torch
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    shape = [(s.field, s.K, s.N, s.width, s.height) for s in renderer.specs]
    fields = [f.n for f in renderer.fields]
    text = json.dumps({"device": dev.name, "arch": getattr(dev, "gcnArchName", ""), "cus": dev.multi_processor_count,
                       "views": shape, "fields": fields, "backward": backward})
    return hashlib.sha1(text.encode()).hexdigest()


def _time_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(renderer, cams: Sequence, backward: bool = True, grid: Optional[Dict[str, Sequence[int]]] = None,
         reps: int = 3, cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Choose and apply the fastest launch shape; returns ``{"tuning", "ms", "cached", "candidates"}``."""
    key = signature(renderer, backward)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        entry = dict(cache[key])
        renderer.set_tuning(**entry["tuning"])
        entry["cached"] = True
        return entry
    renderer.set_cameras(cams)

    def step():
        renderer.forward()
        if backward:
            renderer.backward()

    grid = grid or DEFAULT_GRID
    names = list(grid)
    results = []
    for combo in itertools.product(*(grid[n] for n in names)):
        t = dict(zip(names, combo))
        renderer.set_tuning(**t)
        ms = _time_ms(step, reps)
        results.append({"tuning": t, "ms": round(ms, 4)})
        if log:
            log(f"[autotune] {t} {ms:.3f} ms")
    best = min(results, key=lambda r: r["ms"])
    renderer.set_tuning(**best["tuning"])
    entry = {"tuning": best["tuning"], "ms": best["ms"], "candidates": results}
    if cache_path:
        cache[key] = entry
        try:  # a read-only install still tunes; it only loses the cache
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, cache_path)
        except OSError as e:
            if log:
                log(f"[autotune] cache not written: {e}")
    entry = dict(entry)
    entry["cached"] = False
    return entry


BUDGET_LADDER = (1 << 26, 1 << 27, 1 << 28, 1 << 29)


def tune_budget(build, cams: Sequence, target_ms: float, budgets: Sequence[int] = BUDGET_LADDER,
                backward: bool = True, reps: int = 3, cache_path: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Choose the cascade texel budget of a batch by measurement: the largest budget of the ladder whose
    batch step (forward, and with ``backward`` the backward pass too; launch shape tuned by ``tune`` at
    each budget) fits ``target_ms``, i.e. the finest cascades the batch affords in its time.  ``build(budget)``
    returns a ``BatchRenderer`` whose views take N from ``texel_budget(..., budget)``.  Returns
    ``{"budget", "renderer", "ms", "curve"}`` (the smallest budget when none fits); every renderer but the
    chosen one is released."""
    import torch
    curve, chosen = [], None
    for budget in sorted(budgets):
        R = build(budget)
        tuned = tune(R, cams, backward=backward, reps=reps, cache_path=cache_path, log=log)
        R.set_cameras(cams)

        def step():
            R.forward()
            if backward:
                R.backward()

        ms = _time_ms(step, reps)
        texels = sum(s.K * s.N * s.N for s in R.specs)
        curve.append({"budget": budget, "texels": texels, "ms": round(ms, 4), "tuning": tuned["tuning"]})
        if log:
            log(f"[autotune] budget 2^{budget.bit_length() - 1}: {texels} texels, {ms:.3f} ms")
        if chosen is None or ms <= target_ms:
            chosen = (budget, R, ms)  # the previous choice's buffers go with its last reference
        else:
            del R
            break  # larger budgets only take longer
        torch.cuda.empty_cache()
    return {"budget": chosen[0], "renderer": chosen[1], "ms": round(chosen[2], 4), "target_ms": target_ms,
            "curve": curve}
