"""The oracle's gradient of the differentiable workload's image loss against
central finite differences of the oracle's own loss (stored in
tests/golden/c4_tiny512_fd.json by make_c4_fd.py; a few probes are recomputed
here so that a change to the oracle or the inputs cannot leave a stale file).

This pins the whole adjoint chain of the oracle (ray root derivative, blend
term, Eq. 2 adjoint for heights and widths) on a realistic frame, beyond the
small-case finite-difference tests."""
import json
import os

import numpy as np
import pytest

from tests import differentiable as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c4_tiny512_fd.json")


@pytest.fixture(scope="module")
def problem():
    return D.build_problem()


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def test_stored_loss_is_current(problem, gold):
    assert problem["loss0"] == pytest.approx(gold["loss"], rel=1e-12)


@pytest.mark.parametrize("which", ["v", "sigma"])
def test_oracle_gradient_matches_stored_fd(problem, gold, which):
    g = problem["gv"] if which == "v" else problem["gs"]
    G = gold[which]
    leaf, fd = np.array(G["leaf"]), np.array(G["fd"])
    assert len(leaf) == 64
    rel = np.abs(g[leaf] - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(g).max())
    assert rel.max() <= 1e-3, rel.max()
    assert np.median(rel) <= 1e-6, np.median(rel)


@pytest.mark.parametrize("which", ["v", "sigma"])
def test_stored_fd_recomputes(problem, gold, which):
    G = gold[which]
    for a in range(3):
        f = D.fd(problem, G["leaf"][a], which, G["eps"][a])
        assert f is not None
        assert f == pytest.approx(G["fd"][a], rel=1e-9, abs=1e-9 * G["grad_inf_norm"])
