"""Pins of the oracle's plain-C form of Eq. 1 / Eq. 2 and its adjoint (``oracle/c/rbf_oracle.c``).

The C form serves the full-size scenes.  It is pinned to the definition
itself (the sum over every leaf, written in NumPy), to closed forms (a
tilted plane on a uniform grid, a constant field) and, for the adjoint, to
central finite differences of its own forward sums.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import adjoint, discretize
from paper_2201_10887_amd import synth


def _leaves_random(depth, p_split, seed, side=512.0):
    struct = synth.random_leaf_structure(depth, p_split, seed)
    rng = np.random.default_rng(seed)
    n = len(struct)
    return synth.leaves_from_structure(struct, side, rng.uniform(-50, 250, n), rng.uniform(0.8, 1.6, n))


@settings(max_examples=12, deadline=None)
@given(seed=st.integers(0, 10_000), depth=st.integers(2, 6), p=st.floats(0.2, 0.8),
       cutoff=st.sampled_from([2.5, 3.0, 3.5]), basis=st.sampled_from(discretize.BASES))
def test_c_form_equals_all_leaves(seed, depth, p, cutoff, basis):
    """Every leaf with w > 0 and no other: the C form equals the brute-force sum over all leaves."""
    L = _leaves_random(depth, p, seed)
    pts = np.random.default_rng(seed + 1).uniform(0, 512.0, (400, 2))
    a, sa = discretize.rbf_bruteforce(pts, L, cutoff, basis=basis)
    b, sb = discretize.rbf_evaluate_c(L, cutoff, pts, basis, threads=3)
    assert np.abs(a - b).max() <= 1e-12 * 300 and np.allclose(sa, sb, rtol=1e-12, atol=0)


def test_c_form_equals_all_leaves_on_tiny_scene(tiny_scene):
    s = tiny_scene
    rng = np.random.default_rng(4)
    pts = np.concatenate([rng.uniform(0, s.work.side, (3000, 2)),
                          [[0.0, 0.0], [s.work.side, s.work.side], [0.0, s.work.side], [17.0, 0.0]]])
    a, sa = discretize.rbf_bruteforce(pts, s.leaves, s.work.cutoff)
    b, sb = discretize.rbf_evaluate_c(s.leaves, s.work.cutoff, pts, threads=4)
    assert np.abs(a - b).max() < 1e-10 and np.allclose(sa, sb, rtol=1e-12, atol=0)


@pytest.mark.parametrize("basis", discretize.BASES)
def test_c_form_reproduces_a_tilted_plane(basis):
    """Symmetric neighbourhoods on a uniform grid cancel first moments: the plane exactly."""
    level, side, sigma, cutoff = 5, 640.0, 1.0, 3.5
    c = side / 2 ** level
    struct = [(level, i, j) for j in range(2 ** level) for i in range(2 ** level)]
    a, b, c0 = 0.375, -0.1875, 12.5
    xs = (np.array([s[1] for s in struct]) + 0.5) * c
    ys = (np.array([s[2] for s in struct]) + 0.5) * c
    L = synth.leaves_from_structure(struct, side, a * xs + b * ys + c0, np.full(len(struct), sigma))
    R = cutoff * sigma * c
    g = np.arange(0.0, side + 1e-9, c / 2)
    px, py = np.meshgrid(g, g)
    pts = np.stack([px.ravel(), py.ravel()], axis=1)
    pts = pts[np.all((pts > R + c) & (pts < side - R - c), axis=1)]
    v, _ = discretize.rbf_evaluate_c(L, cutoff, pts, basis)
    assert np.abs(v - (a * pts[:, 0] + b * pts[:, 1] + c0)).max() < 1e-9


def test_c_form_constant_field():
    L = _leaves_random(5, 0.5, 9)
    L["v"] = np.full(len(L["x"]), 123.25, np.float32)
    pts = np.random.default_rng(2).uniform(0, 512.0, (1000, 2))
    v, s0 = discretize.rbf_evaluate_c(L, 3.0, pts)
    assert np.all(s0 > 0) and np.abs(v - 123.25).max() < 1e-12


def test_c_discretize_equals_numpy_discretize(tiny_scene):
    s = tiny_scene
    for cas, ref in zip(s.cascades, s.tex64):
        got = discretize.discretize_c(cas, s.leaves, s.dom, s.work.cutoff, threads=2)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin)
        assert np.abs(got[fin] - ref[fin]).max() < 1e-10


@pytest.mark.parametrize("basis", discretize.BASES)
def test_c_adjoint_matches_finite_differences(basis):
    """d/dv_j and d/dsigma_j of sum_s g_s v(p_s) by central differences of the C forward form."""
    L = _leaves_random(4, 0.5, 21)
    cutoff = 3.0
    rng = np.random.default_rng(5)
    pts = rng.uniform(40.0, 470.0, (60, 2))
    g = rng.normal(0, 1, len(pts))

    arrs = discretize._leaf_arrays(L)
    n = len(arrs[0])
    gv, gs = np.zeros(n), np.zeros(n)
    lib = discretize._c_lib()
    px, py = np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1])
    assert lib.oracle_rbf_adjoint(n, *(discretize._p(a) for a in arrs), cutoff, discretize.BASES.index(basis), len(pts),
                                  discretize._p(px), discretize._p(py), discretize._p(g), discretize._p(gv),
                                  discretize._p(gs)) == 0

    def loss(Lx):
        v, _ = discretize.rbf_evaluate_c(Lx, cutoff, pts, basis)
        return float(np.dot(g, v))

    touched = np.nonzero(gv)[0]
    for j in rng.choice(touched, 12, replace=False):
        for key, grad, eps in (("v", gv, 1e-3), ("sigma", gs, 1e-6)):
            Lp = {k: np.asarray(a, np.float64).copy() for k, a in L.items()}
            Lm = {k: np.asarray(a, np.float64).copy() for k, a in L.items()}
            Lp[key][j] += eps
            Lm[key][j] -= eps
            fd = (loss(Lp) - loss(Lm)) / (2 * eps)
            assert abs(fd - grad[j]) <= 1e-5 * max(abs(fd), 1e-3), (key, j, fd, grad[j])


def test_c_adjoint_equals_numpy_adjoint(tiny_scene):
    s = tiny_scene
    K, N = len(s.cascades), s.cascades[0].n
    rng = np.random.default_rng(8)
    gtex = np.zeros((K, N, N))
    for k in range(K):
        jj, ii = np.nonzero(np.isfinite(s.tex64[k]))
        pick = rng.choice(len(jj), 500, replace=False)
        gtex[k][jj[pick], ii[pick]] = rng.normal(0, 1, 500)
    gv_ref, gs_ref = adjoint.leaf_gradients(s.cascades, s.field, s.dom, gtex)
    gv, gs = adjoint.leaf_gradients_c(s.cascades, s.leaves, s.work.cutoff, s.dom, gtex)
    assert np.abs(gv - gv_ref).max() <= 1e-12 * np.abs(gv_ref).max()
    assert np.abs(gs - gs_ref).max() <= 1e-12 * np.abs(gs_ref).max()
