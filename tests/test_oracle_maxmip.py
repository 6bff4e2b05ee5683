"""Pin of the oracle maximum mipmap against brute-force footprint maxima."""
import numpy as np
import pytest

from oracle import maxmip


@pytest.mark.parametrize("N,seed,frac", [(2, 0, 0.0), (8, 1, 0.2), (16, 2, 0.5), (32, 3, 0.05)])
def test_maxmip_bruteforce(N, seed, frac):
    rng = np.random.default_rng(seed)
    tex = rng.normal(100.0, 30.0, (N, N))
    tex[rng.random((N, N)) < frac] = -np.inf
    levels = maxmip.maxmip(tex)
    assert len(levels) == int(np.log2(N)) + 1
    assert sum(m.size for m in levels) == (4 * N * N - 1) // 3
    for l, m in enumerate(levels):
        s = 2 ** l
        assert m.shape == (N // s, N // s)
        for j in range(N // s):
            for i in range(N // s):
                best = -np.inf
                for cj in range(j * s, (j + 1) * s):
                    for ci in range(i * s, (i + 1) * s):
                        if ci >= N - 1 or cj >= N - 1:
                            continue
                        corners = [tex[cj, ci], tex[cj, ci + 1], tex[cj + 1, ci], tex[cj + 1, ci + 1]]
                        if all(np.isfinite(corners)):
                            best = max(best, max(corners))
                assert m[j, i] == best
    flat = maxmip.flatten(levels)
    assert flat.shape == ((4 * N * N - 1) // 3,) and flat[0] == levels[0][0, 0] and flat[-1] == levels[-1][0, 0]
