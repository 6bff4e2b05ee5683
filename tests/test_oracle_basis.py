"""Pins of the oracle's second basis (Wendland's compactly supported C2 function in Eq. 2's place).

What fixes it independently of its formula: the weight is 1 at the centre, vanishes with its first
two derivatives at the support radius, and integrates to pi R^2 / 7 over the plane (among
(1 - u)^4 (a u + 1) that integral holds for a = 4 only); the width derivative matches finite
differences of the weight; Eq. 2 by range queries equals the sum over every leaf; constants and
planes are reproduced on a uniform grid (symmetric neighbourhoods).
"""
import math

import numpy as np
import pytest

from oracle import discretize
from paper_2201_10887_amd import synth

K, C, SG = 3.5, 20.0, 1.3
R = K * SG * C


def _w(r, basis="wendland", sigma=SG):
    r = np.atleast_1d(np.asarray(r, np.float64))
    return discretize.weights(np.zeros((1, 2)), r, np.zeros_like(r), np.full_like(r, C), np.full_like(r, sigma), K,
                              basis)[0]


def test_centre_and_support():
    assert _w(0.0)[0] == 1.0
    r = np.linspace(0.0, 1.2 * R, 4001)
    w = _w(r)
    inside = r < R
    assert np.all(w[inside] > 0) and np.all(w[~inside] == 0) and np.all(np.diff(w) <= 0)


def test_smooth_at_the_support_edge():
    # first and second derivatives (central differences) go to 0 at r -> R from inside
    for h in (1e-2 * R, 1e-3 * R):
        r = R - 4 * h
        d1 = (_w(r + h) - _w(r - h))[0] / (2 * h)
        d2 = (_w(r + h) - 2 * _w(r) + _w(r - h))[0] / (h * h)
        # (1 - u)^4 behaviour: d1 ~ (4h)^3, d2 ~ (4h)^2 up to constants of order 1 / R^k
        assert abs(d1) * R < 1e3 * (4 * h / R) ** 3 and abs(d2) * R * R < 1e3 * (4 * h / R) ** 2
    # and the weight itself vanishes like the fourth power: halving the distance divides by ~16
    a, b = _w(R - 1e-3 * R)[0], _w(R - 5e-4 * R)[0]
    assert 15.5 < a / b < 16.5


def test_integral_over_the_plane():
    h = R / 400
    g = (np.arange(-400, 400) + 0.5) * h
    X, Y = np.meshgrid(g, g)
    r = np.hypot(X, Y).ravel()
    total = 0.0
    for a in range(0, len(r), 100_000):
        total += _w(r[a:a + 100_000]).sum()
    total *= h * h
    assert math.isclose(total, math.pi * R * R / 7.0, rel_tol=2e-5)


@pytest.mark.parametrize("basis", discretize.BASES)
def test_width_derivative_matches_finite_differences(basis):
    r = np.linspace(0.02 * R, 0.98 * R, 37)
    eps = 1e-6 * SG
    fd = (_w(r, basis, SG + eps) - _w(r, basis, SG - eps)) / (2 * eps)
    q = r / (SG * C)
    an = discretize.basis_dweight_dsigma(q, np.full_like(q, SG), K, basis)
    assert np.abs(fd - an).max() <= 1e-7 * np.abs(an).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_range_query_equals_all_leaves(seed):
    struct = synth.random_leaf_structure(5, 0.5, seed)
    rng = np.random.default_rng(seed)
    n = len(struct)
    L = synth.leaves_from_structure(struct, 512.0, rng.uniform(-50, 250, n), rng.uniform(0.8, 1.6, n))
    pts = np.random.default_rng(seed + 1).uniform(0, 512.0, (400, 2))
    a, sa = discretize.rbf_bruteforce(pts, L, 3.0, basis="wendland")
    b, sb = discretize.RBFField(L, 3.0, "wendland").evaluate(pts)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * 300) and np.allclose(sa, sb, rtol=1e-12, atol=0)


@pytest.mark.parametrize("sigma,cutoff", [(1.0, 3.5), (0.9, 2.0)])
def test_plane_and_constant_reproduced_on_uniform_grid(sigma, cutoff):
    level, side = 5, 640.0
    c = side / 2 ** level
    struct = [(level, i, j) for j in range(2 ** level) for i in range(2 ** level)]
    xs = (np.array([s[1] for s in struct]) + 0.5) * c
    ys = (np.array([s[2] for s in struct]) + 0.5) * c
    g = np.arange(0.0, side + 1e-9, c / 2)
    px, py = np.meshgrid(g, g)
    pts = np.stack([px.ravel(), py.ravel()], axis=1)
    Rr = cutoff * sigma * c
    pts = pts[np.all((pts > Rr + c) & (pts < side - Rr - c), axis=1)]
    a, b, c0 = 0.375, -0.1875, 12.5
    for vals, ref in ((a * xs + b * ys + c0, a * pts[:, 0] + b * pts[:, 1] + c0),
                      (np.full(len(xs), 7.25), np.full(len(pts), 7.25))):
        L = synth.leaves_from_structure(struct, side, vals, np.full(len(struct), sigma))
        v, _ = discretize.RBFField(L, cutoff, "wendland").evaluate(pts)
        assert np.abs(v - ref).max() < 1e-9


def test_bases_differ_where_expected():
    # same support, different shape: equal zero sets, different weights inside
    r = np.linspace(0.0, 1.1 * R, 500)
    wg, ww = _w(r, "gaussian"), _w(r, "wendland")
    assert np.array_equal(wg > 0, ww > 0)
    assert np.abs(wg - ww)[r < 0.9 * R].max() > 0.02
