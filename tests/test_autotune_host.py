"""Host logic of the batch autotuner (no GPU): the texel budget's N per view, the launch-shape
search and its cache, and the budget choice, with the timing replaced by a seeded cost model."""
import itertools

import pytest

from paper_2201_10887_amd import autotune

VIEWS = [(1920, 1080, 4), (256, 256, 2), (1280, 720, 3), (512, 512, 2), (1920, 1080, 2), (300, 200, 4)]


def test_texel_budget_unbounded_takes_the_image_side():
    ns = autotune.texel_budget(VIEWS, 1 << 40)
    # one texel per pixel of the larger side, a power of two, clamped to [256, 2048]
    assert ns == [2048, 256, 2048, 512, 2048, 512]


@pytest.mark.parametrize("budget", [1 << 20, 1 << 24, 1 << 25, 1 << 26, 1 << 27])
def test_texel_budget_fits_by_halving_the_largest_first(budget):
    ns = autotune.texel_budget(VIEWS, budget)
    full = autotune.texel_budget(VIEWS, 1 << 40)
    total = sum(k * n * n for (_, _, k), n in zip(VIEWS, ns))
    assert all(n & (n - 1) == 0 and 256 <= n <= f for n, f in zip(ns, full))
    if total > budget:  # only when every view is already at the floor
        assert all(n == 256 for n in ns)
    else:
        # largest first: no view was halved while a larger one was left (ties go to the earlier view)
        halved = [a for a in range(len(ns)) if ns[a] < full[a]]
        for a in halved:
            assert all(ns[b] <= 2 * ns[a] for b in range(len(ns))), (ns, a)
        # and it stops as soon as the budget fits: undoing the last halving overflows it
        if halved:
            last = max(halved, key=lambda a: (-ns[a], a))
            undo = list(ns)
            undo[last] *= 2
            assert sum(k * n * n for (_, _, k), n in zip(VIEWS, undo)) > budget


def test_texel_budget_is_monotone():
    prev = None
    for e in range(18, 30):
        ns = autotune.texel_budget(VIEWS, 1 << e)
        if prev is not None:
            assert all(a >= b for a, b in zip(ns, prev))
        prev = ns


class StubRenderer:
    """Records the launch shapes set; the cost model reads the current one."""

    def __init__(self, best):
        self.best = best
        self.tuning = None
        self.calls = []

    def set_tuning(self, **t):
        self.tuning = dict(t)
        self.calls.append(dict(t))

    def set_cameras(self, cams):
        pass

    def forward(self):
        pass

    def backward(self):
        pass

    def cost(self):
        # 10 ms at the best shape, plus 1 ms per field that differs
        return 10.0 + sum(self.tuning[k] != v for k, v in self.best.items())


@pytest.fixture
def stubbed(monkeypatch):
    state = {}

    def fake_time(step, reps):
        return state["renderer"].cost()

    monkeypatch.setattr(autotune, "_time_ms", fake_time)
    monkeypatch.setattr(autotune, "signature", lambda r, backward: "stub-" + repr(sorted(r.best.items())))
    return state


def test_tune_finds_and_applies_the_fastest_shape_and_caches_it(stubbed, tmp_path):
    grid = {k: v for k, v in autotune.DEFAULT_GRID.items()}
    best = {k: v[-1] for k, v in grid.items()}
    best["ray_grain"] = 8
    R = StubRenderer(best)
    stubbed["renderer"] = R
    cache = str(tmp_path / "tune.json")
    out = autotune.tune(R, [], backward=True, grid=grid, cache_path=cache)
    assert out["tuning"] == best and out["ms"] == 10.0 and not out["cached"]
    assert R.tuning == best
    n = 1
    for v in grid.values():
        n *= len(v)
    assert len(out["candidates"]) == n
    assert [c["tuning"] for c in out["candidates"]] == [dict(zip(grid, combo))
                                                         for combo in itertools.product(*grid.values())]
    # a second call with the same batch shape reads the cache and times nothing
    R2 = StubRenderer(best)
    stubbed["renderer"] = R2
    out2 = autotune.tune(R2, [], backward=True, grid=grid, cache_path=cache)
    assert out2["cached"] and out2["tuning"] == best and R2.calls == [best]


def test_tune_budget_takes_the_largest_budget_that_fits(stubbed):
    made = []

    class Budgeted(StubRenderer):
        def __init__(self, budget):
            super().__init__({"disc_grain": 8})
            self.budget = budget
            self.specs = [type("S", (), {"K": 2, "N": 256})()]

        def cost(self):
            return self.budget / (1 << 24) * 4.0  # 16, 32, 64, 128 ms over the ladder

    def build(budget):
        R = Budgeted(budget)
        made.append(budget)
        stubbed["renderer"] = R
        return R

    grid = {"disc_grain": (8, 16)}
    real_tune = autotune.tune
    tune = lambda R, cams, backward, reps, cache_path, log: real_tune(R, cams, backward, grid, reps, None, log)
    autotune_tune = autotune.tune
    try:
        autotune.tune = tune
        out = autotune.tune_budget(build, [], 40.0)
        assert out["budget"] == 1 << 27 and out["ms"] == 32.0
        assert made == [1 << 26, 1 << 27, 1 << 28]  # the first budget over the target ends the ladder
        assert [c["ms"] for c in out["curve"]] == [16.0, 32.0, 64.0]
        made.clear()
        out = autotune.tune_budget(build, [], 5.0)  # nothing fits: the smallest budget
        assert out["budget"] == 1 << 26 and made == [1 << 26, 1 << 27]
    finally:
        autotune.tune = autotune_tune
