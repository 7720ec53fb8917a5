"""Scheduling study of the paper's load-balancing analysis (oracle).

TEST INFRASTRUCTURE ONLY.

list_schedule: Step 3 of Algorithm PH (and of its improved form, Section 3.3): the jobs are
taken in a given order and each is given to the currently least-loaded processor. Ties between
equally loaded processors are broken by the lowest processor index (the paper does not say;
any rule gives the same makespan distribution, and one fixed rule makes results comparable).
The makespan is the largest processor load; the parallel efficiency on k processors is
sum(times) / (k * makespan).

kendall_tau: Kendall's rank correlation as the paper defines it (Section 3.2): for every pair
i < j the scores a_ij = sign(x_j - x_i) and b_ij = sign(y_j - y_i) (zero for a tie), S = the
sum of a_ij * b_ij over the pairs, and with ties (the equations for tied ranks)
tau = S / sqrt((n(n-1)/2 - T) (n(n-1)/2 - U)), T and U the sums of t(t-1)/2 over the groups of
equal x and of equal y. Under independence tau is close to normal with mean 0 and variance
2(2n+5) / (9n(n-1)) (the variance the paper quotes), which gives the normal score and a
two-sided p-value. Plain O(n^2) loops: for inputs of a few thousand at most.
"""
from __future__ import annotations

import math

import numpy as np


def list_schedule(times, order, machines: int) -> tuple[int, list[int]]:
    """(makespan, loads) of list scheduling `times` in `order` on `machines` processors."""
    if machines < 1:
        raise ValueError("machines must be >= 1")
    order = [int(k) for k in order]
    if sorted(order) != list(range(len(times))):
        raise ValueError("order must be a permutation")
    loads = [0] * machines
    for k in order:
        best = 0
        for i in range(1, machines):
            if loads[i] < loads[best]:
                best = i
        loads[best] += int(times[k])
    return max(loads), loads


def efficiency(times, makespan: int, machines: int) -> float:
    return float(sum(int(t) for t in times)) / (machines * makespan)


def _tied_pairs(v) -> int:
    _, counts = np.unique(np.asarray(v), return_counts=True)
    return int(sum(int(c) * (int(c) - 1) // 2 for c in counts))


def kendall_tau(x, y) -> tuple[float, float, float]:
    """(tau with tie correction, normal score, two-sided p-value) of x and y."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    if n < 2 or y.size != n:
        raise ValueError("two sequences of equal length >= 2 expected")
    s = 0
    for i in range(n - 1):   # one row of pairs (i, j > i) at a time
        a = np.sign(x[i + 1:] - x[i])
        b = np.sign(y[i + 1:] - y[i])
        s += int(np.sum(a * b))
    n0 = n * (n - 1) // 2
    t, u = _tied_pairs(x), _tied_pairs(y)
    if t == n0 or u == n0:
        raise ValueError("every pair is tied in one of the rankings")
    tau = s / math.sqrt((n0 - t) * (n0 - u))
    z = tau / math.sqrt(2.0 * (2 * n + 5) / (9.0 * n * (n - 1)))
    return tau, z, math.erfc(abs(z) / math.sqrt(2.0))


def opt_makespan_brute(times, machines: int) -> int:
    """The optimal makespan by trying every assignment (tiny inputs only)."""
    times = [int(t) for t in times]
    best = sum(times)

    def rec(k, loads):
        nonlocal best
        if max(loads) >= best:
            return
        if k == len(times):
            best = max(loads)
            return
        seen = set()
        for i in range(machines):   # machines with equal loads are interchangeable
            if loads[i] in seen:
                continue
            seen.add(loads[i])
            loads[i] += times[k]
            rec(k + 1, loads)
            loads[i] -= times[k]

    rec(0, [0] * machines)
    return best
