"""The permanental polynomial per(xI - A) (the paper's application section) in exact integers
(oracle).

TEST INFRASTRUCTURE ONLY.

Two independent routes, both from the definition of the permanent (eq. 1):
* by principal sub-matrices: expanding per(xI - A) over the rows that take the diagonal x,
  the coefficient of x^k is (-1)^(n-k) times the sum of per(A[S, S]) over the index sets S of
  size n - k (small n only: 2^n sub-matrices);
* by evaluation: per(xI - A) at the n + 1 integers x = 0..n (signed entries; the frontier
  dynamic programme, which accepts any integers), then Lagrange interpolation in exact
  rational arithmetic.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

from .permanent import per_dp, per_ryser


def perpoly_subsets(A) -> list[int]:
    """Coefficients c_0..c_n (c_k of x^k) from the principal sub-matrices (n <= 14)."""
    A = np.asarray(A, dtype=object)
    n = A.shape[0]
    c = [0] * (n + 1)
    for s in range(n + 1):
        total = 0
        for S in itertools.combinations(range(n), s):
            total += per_ryser(A[np.ix_(S, S)]) if s else 1
        c[n - s] = (-1) ** s * total
    return c


def perpoly_interpolate(A) -> list[int]:
    """Coefficients c_0..c_n from per(xI - A) at x = 0..n and Lagrange interpolation."""
    A = np.asarray(A, dtype=object)
    n = A.shape[0]
    xs = list(range(n + 1))
    ys = []
    for x in xs:
        M = -A.copy()
        for i in range(n):
            M[i, i] += x
        ys.append(per_dp(M.tolist()))
    return interpolate(ys)


def interpolate(ys) -> list[int]:
    """Integer coefficients (low to high) of the polynomial of degree <= n through (x, ys[x]),
    x = 0..n, by Lagrange's formula in exact rationals (ArithmeticError if not integral)."""
    n = len(ys) - 1
    xs = list(range(n + 1))
    coeffs = [Fraction(0)] * (n + 1)
    for i, (xi, yi) in enumerate(zip(xs, ys)):
        # basis polynomial prod_{j != i} (x - x_j) / (x_i - x_j), coefficients low to high
        basis = [Fraction(1)]
        denom = 1
        for j, xj in enumerate(xs):
            if j == i:
                continue
            basis = [Fraction(0)] + basis
            for t in range(len(basis) - 1):
                basis[t] -= xj * basis[t + 1]
            denom *= xi - xj
        for t in range(n + 1):
            coeffs[t] += yi * basis[t] / denom
    out = []
    for v in coeffs:
        if v.denominator != 1:
            raise ArithmeticError("interpolated coefficient is not an integer")
        out.append(int(v))
    return out
