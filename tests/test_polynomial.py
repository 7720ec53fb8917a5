"""The permanental polynomial per(xI - A): the oracle's two routes against each other and
against closed forms, then the library (GPU) against the oracle."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import per_brute
from oracle.polynomial import interpolate, perpoly_interpolate, perpoly_subsets


@pytest.fixture(scope="module")
def hostlib():
    """The library's host-side calls (no GPU needed for these)."""
    import paper_1112_6072_amd as hp
    return hp


def test_routes_agree_on_random_integer_matrices():
    rng = np.random.default_rng(4)
    for n in (1, 2, 3, 5, 7):
        A = rng.integers(0, 4, (n, n))
        assert perpoly_subsets(A) == perpoly_interpolate(A)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_all_ones_closed_form(n):
    """per(xI - J) = sum_s (-1)^s C(n, s) s! x^(n-s): every principal sub-matrix of J of order s
    has permanent s!."""
    J = np.ones((n, n), dtype=np.int64)
    want = [0] * (n + 1)
    for s in range(n + 1):
        want[n - s] = (-1) ** s * math.comb(n, s) * math.factorial(s)
    assert perpoly_subsets(J) == want
    assert perpoly_interpolate(J) == want


def test_low_order_coefficients():
    """c_n = 1, c_(n-1) = -tr A, c_(n-2) = sum_(i<j) (a_ii a_jj + a_ij a_ji), c_0 = (-1)^n per(A)."""
    rng = np.random.default_rng(8)
    for n in (3, 4, 6):
        A = rng.integers(0, 5, (n, n))
        c = perpoly_interpolate(A)
        assert c[n] == 1
        assert c[n - 1] == -int(np.trace(A))
        assert c[n - 2] == sum(int(A[i, i] * A[j, j] + A[i, j] * A[j, i]) for i in range(n) for j in range(i + 1, n))
        assert c[0] == (-1) ** n * per_brute(A)
    assert perpoly_interpolate(np.zeros((4, 4), dtype=np.int64)) == [0, 0, 0, 0, 1]


def test_native_interpolation_matches_oracle(hostlib):
    """The host step of the library: exact interpolation against Lagrange's formula."""
    rng = np.random.default_rng(31)
    for n in (0, 1, 2, 5, 12, 30):
        coeffs = [int(v) for v in rng.integers(0, 10 ** 6, n + 1)]
        coeffs[-1] = coeffs[-1] or 1
        ys = [sum(c * x ** k for k, c in enumerate(coeffs)) for x in range(n + 1)]
        assert interpolate(ys) == coeffs
        assert hostlib.polynomial_interpolate(ys) == coeffs
        alt = hostlib.polynomial_interpolate(ys, alternate=True)
        assert alt == [(-1) ** (n - k) * c for k, c in enumerate(coeffs)]
    # large values: per(xI + A) of a cubic graph on 34 vertices reaches about 2^175
    ys = [(x + 3) ** 34 for x in range(35)]
    want = interpolate(ys)
    assert hostlib.polynomial_interpolate(ys) == want
    # x(x-1)/2 has no integer coefficients
    with pytest.raises(hostlib.HpermError):
        hostlib.polynomial_interpolate([0, 0, 1])


@pytest.mark.gpu
def test_library_matches_oracle(hperm):
    c = hperm.Context()
    try:
        rng = np.random.default_rng(12)
        cases = [np.zeros((0, 0), dtype=np.uint32), np.array([[3]], dtype=np.uint32),
                 rng.integers(0, 4, (8, 8)).astype(np.uint32)]
        cases += [W.random_cubic_matrix(n, s) for n, s in ((10, 1), (16, 2), (24, 0))]
        for A in cases:
            got = c.permanental_polynomial(A)
            want = perpoly_interpolate(A.astype(np.int64))
            assert got == want, A.shape
        # a cubic graph: c_n = 1, c_(n-1) = 0, c_(n-2) = |E|, c_0 = per(A)
        G = W.random_cubic_matrix(24, 0)
        got = c.permanental_polynomial(G)
        assert got[24] == 1 and got[23] == 0 and got[22] == 36
        assert got[0] == c.permanent(G)
        # per(nI + A) of a cubic graph on 40 vertices exceeds the supported bound
        with pytest.raises(hperm.HpermError) as e:
            c.permanental_polynomial(W.random_cubic_matrix(40, 0))
        assert e.value.status == -2
    finally:
        c.close()
