"""The regression of the paper's Section 3.1 (eqs. 4-6): the oracle (oracle/regression.py)
pinned against brute force and closed forms, and the library's host calls (hperm_ols,
hperm_stepwise, hperm_matrix_invariants) against the oracle."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle.regression import determinant_abs, invariants, ols, r_squared, stepwise


@pytest.fixture(scope="module")
def hperm():
    """The library's host-side calls (no GPU needed for these)."""
    import paper_1112_6072_amd as hp
    return hp


def det_leibniz(B) -> int:
    """The defining sum over permutations with their signs (small n only)."""
    n = len(B)
    total = 0
    for p in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if p[i] > p[j])
        term = 1
        for i in range(n):
            term *= int(B[i][p[i]])
        total += -term if inv & 1 else term
    return total


def test_determinant_against_leibniz_and_laws():
    rng = np.random.default_rng(5)
    for n in range(1, 7):
        for _ in range(6):
            B = rng.integers(0, 5, size=(n, n))
            B[rng.random((n, n)) < 0.4] = 0
            assert determinant_abs(B) == abs(det_leibniz(B))
    assert determinant_abs(np.eye(9, dtype=int)) == 1
    assert determinant_abs(np.ones((4, 4), dtype=int)) == 0
    P = np.eye(7, dtype=int)[[3, 0, 6, 1, 5, 2, 4]]
    assert determinant_abs(P) == 1
    B = rng.integers(0, 4, size=(5, 5))
    C = B.copy()
    C[2] *= 3   # scaling a row scales |det|
    assert determinant_abs(C) == 3 * determinant_abs(B)


def test_invariants_by_hand():
    A = np.array([[1, 2], [0, 3]])
    # |det| 3; S = 3; row sums 3, 3 (variance 0); column sums 1, 5 (mean 3, variance 4)
    assert invariants(A) == (3, 3, 0.0, 4.0)
    G = W.random_cubic_matrix(24, 1)   # every row and column sums to 3
    d, s, v1, v2 = invariants(G)
    assert s == 72 and v1 == 0.0 and v2 == 0.0


def test_r_squared_closed_forms():
    rng = np.random.default_rng(2)
    x = rng.normal(size=300)
    y = 1.5 - 0.7 * x + rng.normal(size=300)
    coef, r2, rss = ols(x[:, None], y)
    # one regressor: R^2 is the squared Pearson correlation
    assert r2 == pytest.approx(np.corrcoef(x, y)[0, 1] ** 2, rel=1e-12)
    # with an intercept the printed definition equals 1 - RSS / TSS
    assert r2 == pytest.approx(1 - rss / ((y - y.mean()) ** 2).sum(), rel=1e-12)
    # an exact linear relation is fitted exactly
    X = rng.normal(size=(50, 3))
    c, r2e, _ = ols(X, 4 + X @ np.array([1.0, -2.0, 0.5]))
    assert np.allclose(c, [4, 1, -2, 0.5]) and r2e == pytest.approx(1.0)
    assert r_squared(y, np.full_like(y, y.mean())) == 0.0


def test_stepwise_selects_the_planted_factors():
    rng = np.random.default_rng(11)
    X = rng.normal(size=(400, 5))
    y = 3 + 2 * X[:, 0] + 0.1 * rng.normal(size=400)
    assert stepwise(X, y) == [0]
    # a weaker second factor enters after the stronger one (partial F far above 4)
    y2 = X[:, 2] + 0.3 * X[:, 4] + rng.normal(size=400)
    assert stepwise(X, y2) == [2, 4]
    # pure noise: nothing enters... or at most a chance factor; with this seed nothing
    assert stepwise(X, rng.normal(size=400)) == []


def test_library_regression_equals_oracle(hperm):
    rng = np.random.default_rng(3)
    for n, k in ((30, 1), (200, 5), (1000, 3)):
        X = rng.normal(size=(n, k)) * rng.uniform(0.1, 1e6, size=k)   # columns on very different scales
        y = X @ rng.normal(size=k) + 7 + rng.normal(size=n) * 1e3
        c_or, r2_or, _ = ols(X, y)
        c_lib, r2_lib = hperm.ols(X, y)
        assert r2_lib == pytest.approx(r2_or, rel=1e-9)
        assert np.allclose(c_lib, c_or, rtol=1e-7, atol=1e-9 * np.abs(c_or).max())
        assert hperm.stepwise(X, y) == stepwise(X, y)
    with pytest.raises(hperm.HpermError):
        hperm.ols(np.ones((10, 1)), np.arange(10.0))   # a constant column


def test_library_invariants_equal_oracle(hperm):
    for seed, n in enumerate((3, 8, 14, 20, 24)):
        A = W.random_sparse_int_matrix(n, 4, 40 + seed, 0, 5)
        d, s, v1, v2 = hperm.matrix_invariants(A)
        do, so, v1o, v2o = invariants(A)
        assert s == so and v1 == pytest.approx(v1o, rel=1e-15, abs=0) and v2 == pytest.approx(v2o, rel=1e-15, abs=0)
        assert d == pytest.approx(float(do), rel=1e-12, abs=0)
    B = W.random_01_matrix(20, 80, 1)
    assert int(B.sum()) == 80
    assert hperm.matrix_invariants(np.ones((5, 5), np.uint32))[0] == 0.0
