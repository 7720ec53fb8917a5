"""Linear regression of sub-matrix times on matrix invariants (oracle).

TEST INFRASTRUCTURE ONLY.

The paper (Section 3.1, eqs. 4-6, Table T1) regresses the computational time T of H_per on
five invariants of each matrix B:
  P    = per(B);
  |D|  = |det(B)|;
  S    = the number of nonzeros of B;
  V1   = the variance of the row sums of B;
  V2   = the variance of the column sums of B;
with the model T = a0 + a1 P + a2 |D| + a3 S + a4 V1 + a5 V2 (eq. 4), scores the fit by the
coefficient of determination R^2 = sum (yhat_i - ybar)^2 / sum (y_i - ybar)^2 (the definition it
prints), and keeps the significant factors by stepwise regression (eq. 6).

Readings (the paper is silent on them):
  * the variances are population variances (divide by the number of lines);
  * the sums are sums of the entries (for the paper's 0-1 matrices, nonzero counts);
  * stepwise regression is Efroymson's procedure with an F-to-enter of 4.0 and an F-to-remove
    of 3.9: starting from the intercept alone, the candidate whose partial F is largest enters
    while that F exceeds 4.0; after each entry, the model variable whose partial F is smallest
    leaves while that F is below 3.9.

Functions: determinant_abs (exact, by fraction-free elimination in Python integers),
invariants, ols (numpy least squares), r_squared (the printed definition), stepwise.
"""
from __future__ import annotations

import numpy as np


def determinant_abs(B) -> int:
    """|det B| exactly: Bareiss' fraction-free Gaussian elimination in Python integers."""
    a = [[int(x) for x in row] for row in B]
    n = len(a)
    if n == 0:
        return 1
    sign, prev = 1, 1
    for k in range(n - 1):
        if a[k][k] == 0:   # swap in a row with a nonzero pivot
            r = next((i for i in range(k + 1, n) if a[i][k] != 0), None)
            if r is None:
                return 0
            a[k], a[r] = a[r], a[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                a[i][j] = (a[i][j] * a[k][k] - a[i][k] * a[k][j]) // prev
        prev = a[k][k]
    return abs(sign * a[n - 1][n - 1])


def invariants(B) -> tuple[int, int, float, float]:
    """(|D|, S, V1, V2) of an integer matrix B (readings above)."""
    B = np.asarray(B, dtype=np.int64)
    rows = B.sum(axis=1).astype(np.float64)
    cols = B.sum(axis=0).astype(np.float64)
    return (determinant_abs(B), int(np.count_nonzero(B)),
            float(((rows - rows.mean()) ** 2).mean()), float(((cols - cols.mean()) ** 2).mean()))


def r_squared(y, yhat) -> float:
    """The paper's coefficient of determination: sum (yhat - ybar)^2 / sum (y - ybar)^2."""
    y = np.asarray(y, dtype=np.float64)
    yhat = np.asarray(yhat, dtype=np.float64)
    ybar = y.mean()
    return float(((yhat - ybar) ** 2).sum() / ((y - ybar) ** 2).sum())


def ols(X, y) -> tuple[np.ndarray, float, float]:
    """Least-squares fit of y on the columns of X with an intercept: (coefficients a0..ak,
    R^2, residual sum of squares)."""
    X = np.asarray(X, dtype=np.float64).reshape(len(y), -1)
    y = np.asarray(y, dtype=np.float64)
    A = np.hstack([np.ones((len(y), 1)), X])
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    yhat = A @ coef
    return coef, r_squared(y, yhat), float(((y - yhat) ** 2).sum())


def _rss(X, y, cols) -> float:
    if not cols:
        y = np.asarray(y, dtype=np.float64)
        return float(((y - y.mean()) ** 2).sum())
    return ols(np.asarray(X, dtype=np.float64)[:, cols], y)[2]


def stepwise(X, y, f_enter: float = 4.0, f_remove: float = 3.9) -> list[int]:
    """Efroymson's stepwise selection (reading above): the chosen columns of X, in entry order."""
    X = np.asarray(X, dtype=np.float64)
    n, k = X.shape
    model: list[int] = []
    for _ in range(4 * k):   # each pass enters or removes one variable; cycles are impossible
        rss = _rss(X, y, model)
        best, best_f = None, f_enter
        for j in range(k):
            if j in model or n - len(model) - 2 <= 0:
                continue
            r = _rss(X, y, model + [j])
            if r <= 0:
                f = float("inf")
            else:
                f = (rss - r) / (r / (n - len(model) - 2))
            if f > best_f:
                best, best_f = j, f
        if best is None:
            break
        model.append(best)
        while len(model) > 1:
            rss = _rss(X, y, model)
            worst, worst_f = None, f_remove
            for j in model:
                rest = [c for c in model if c != j]
                f = (_rss(X, y, rest) - rss) / (rss / (n - len(model) - 1)) if rss > 0 else float("inf")
                if f < worst_f:
                    worst, worst_f = j, f
            if worst is None:
                break
            model.remove(worst)
    return model
