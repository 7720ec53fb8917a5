"""Pins for the CPU oracle against facts fixed outside it (closed forms, laws, the paper's values).

Everything here runs on the CPU (no ``gpu`` marker).
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import (choose_line, e2_children, kkl_exponent, kkl_trial, nw_doubled_sum, per_brute,
                    per_dp, per_hybrid, per_nw, per_ryser, splitmix64)
from oracle import native
from oracle import permanent as P


def rand_int(n, seed, hi=5, density=0.6):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, hi + 1, size=(n, n)) * (rng.random((n, n)) < density)).astype(np.int64)


# --------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("k", range(0, 8))
def test_brute_all_ones_is_factorial(k):
    assert per_brute(np.ones((k, k), dtype=int)) == math.factorial(k)


def test_brute_identity_permutation_diagonal():
    assert per_brute(np.eye(6, dtype=int)) == 1
    rng = np.random.default_rng(3)
    p = rng.permutation(7)
    Pm = np.zeros((7, 7), dtype=int)
    Pm[np.arange(7), p] = 1
    assert per_brute(Pm) == 1
    d = [2, 3, 5, 7, 11]
    assert per_brute(np.diag(d)) == 2 * 3 * 5 * 7 * 11


def test_brute_2x2_and_3x3_closed_forms():
    a, b, c, d = 2, 3, 5, 7
    assert per_brute([[a, b], [c, d]]) == a * d + b * c
    M = [[1, 2, 3], [4, 5, 6], [7, 8, 9]]
    # the six permutation products written out
    assert per_brute(M) == 1 * 5 * 9 + 1 * 6 * 8 + 2 * 4 * 9 + 2 * 6 * 7 + 3 * 4 * 8 + 3 * 5 * 7


@pytest.mark.parametrize("k", range(1, 13))
def test_ryser_all_ones_is_factorial(k):
    assert per_ryser(np.ones((k, k), dtype=int)) == math.factorial(k)


# --------------------------------------------------------------------------- routes agree
@pytest.mark.parametrize("seed", range(40))
def test_ryser_nw_hybrid_dp_match_brute(seed):
    n = 1 + seed % 7
    A = rand_int(n, seed)
    b = per_brute(A)
    assert per_ryser(A) == b
    assert per_nw(A) == b
    assert per_hybrid(A) == b
    assert per_dp(A) == b


@pytest.mark.parametrize("seed", range(25))
def test_nw_doubled_sum_identity(seed):
    """V = (-1)^{n-1} 2^{n-1} per(A) for the doubled Nijenhuis-Wilf sum (exact, any integers)."""
    n = 1 + seed % 7
    A = rand_int(n, 100 + seed, hi=9, density=0.7)
    assert nw_doubled_sum(A) == (-1) ** (n - 1) * 2 ** (n - 1) * per_brute(A)


def test_nw_doubled_small_closed_forms():
    assert nw_doubled_sum([[7]]) == 7
    a, b, c, d = 2, 3, 5, 11
    assert nw_doubled_sum([[a, b], [c, d]]) == -2 * (a * d + b * c)


def test_c_ryser_and_c_hper_match_brute():
    mats = [rand_int(1 + s % 8, 500 + s, hi=4, density=0.5) for s in range(60)]
    want = [per_brute(A) for A in mats]
    assert native.ryser_batch(mats, threads=4) == want
    assert native.hper_batch(mats, threads=4) == want


def test_c_ryser_wraps_exactly_at_large_values():
    """J_20: per = 20! ~ 2^61.1, Ryser's intermediate products reach 20^20 ~ 2^86.4 (wrap mod 2^128)."""
    assert native.ryser_batch([np.full((20, 20), 1)])[0] == math.factorial(20)
    # 2*J_16 scales every permutation product by 2^16
    assert native.ryser_batch([np.full((16, 16), 2)])[0] == math.factorial(16) * 2 ** 16


# --------------------------------------------------------------------------- laws
@pytest.mark.parametrize("seed", range(12))
def test_laws_transpose_permutation_scaling(seed):
    n = 5 + seed % 4
    A = rand_int(n, 900 + seed)
    b = per_brute(A)
    rng = np.random.default_rng(seed)
    r, c = rng.permutation(n), rng.permutation(n)
    assert per_dp(A.T) == b
    assert per_dp(A[r][:, c]) == b
    k = int(rng.integers(0, n))
    B = A.copy()
    B[k] *= 3
    assert per_dp(B) == 3 * b


@pytest.mark.parametrize("seed", range(6))
def test_block_diagonal_product(seed):
    A = rand_int(4 + seed % 3, 1300 + seed)
    B = rand_int(3 + seed % 4, 1400 + seed)
    n, m = A.shape[0], B.shape[0]
    C = np.zeros((n + m, n + m), dtype=np.int64)
    C[:n, :n] = A
    C[n:, n:] = B
    assert per_dp(C) == per_brute(A) * per_brute(B)
    assert native.hper_batch([C])[0] == per_brute(A) * per_brute(B)


def test_block_diagonal_of_cubic_graphs():
    A = W.random_cubic_matrix(24, 1)
    B = W.random_cubic_matrix(20, 2)
    C = np.zeros((44, 44), dtype=np.int64)
    C[:24, :24] = A
    C[24:, 24:] = B
    assert native.hper_batch([C])[0] == per_dp(A) * per_dp(B)


# --------------------------------------------------------------------------- expansion (2)
@pytest.mark.parametrize("seed", range(30))
def test_e2_children_sum_to_parent_every_line(seed):
    """Expansion (2) along any row or column preserves the permanent; ceil(k/2) children of order n-1."""
    n = 3 + seed % 5
    A = rand_int(n, 2000 + seed, hi=7, density=0.55)
    b = per_brute(A)
    for kind in ("row", "col"):
        for idx in range(n):
            line = A[idx] if kind == "row" else A[:, idx]
            k = int(np.count_nonzero(line))
            kids = e2_children(A, kind, idx)
            assert len(kids) == (k + 1) // 2
            assert all(len(c) == n - 1 and all(len(r) == n - 1 for r in c) for c in kids)
            assert sum(per_brute(c) for c in kids) == b


def test_e2_cross_weighting_is_required(monkeypatch):
    """Plant the swapped merge a*y1 + b*y2 in the oracle: the identity test must catch it."""
    A = np.array([[2, 3, 0, 0], [1, 0, 4, 0], [0, 5, 1, 2], [3, 0, 0, 1]])
    good = e2_children(A, "row", 0)
    assert sum(per_brute(c) for c in good) == per_brute(A)
    # swapped weights: the first child built as 2*y1 + 3*y2 instead of 2*y2 + 3*y1
    y1, y2 = A[1:, 0], A[1:, 1]
    bad = np.column_stack([2 * y1 + 3 * y2, A[1:, 2], A[1:, 3]])
    assert per_brute(bad) != per_brute(good[0])


def test_choose_line_tie_rule():
    A = np.array([[1, 1, 0], [1, 0, 1], [0, 1, 1]])
    assert choose_line(A) == ("row", 0, 2)
    B = np.array([[1, 1, 0], [1, 1, 0], [1, 1, 1]])
    assert choose_line(B) == ("col", 2, 1)


# --------------------------------------------------------------------------- the paper's values
def test_t12_fixture_sums_to_printed_total():
    total, vals = W.read_c100_subpermanents()
    assert len(vals) == 159 and sorted(vals) == list(range(1, 160))
    assert sum(vals.values()) == total == 149364113290700


@pytest.mark.slow
def test_c100_permanent_matches_paper():
    """per(A(C100)) = 149 364 113 290 700: the paper's appendix total (sum over the 159 jobs)."""
    A = W.adjacency_matrix(W.read_appendix_adjacency("c100"))
    assert per_dp(A) == 149364113290700


def test_c60_appendix_and_truncated_icosahedron_agree():
    import networkx as nx
    app = W.read_appendix_adjacency("c60")
    ti = W.truncated_icosahedron()
    G1 = nx.Graph([(u, v) for u, nb in enumerate(app) for v in nb])
    G2 = nx.Graph([(u, v) for u, nb in enumerate(ti) for v in nb])
    assert nx.is_isomorphic(G1, G2)
    A1, A2 = W.adjacency_matrix(app), W.adjacency_matrix(ti)
    assert native.hper_batch([A1, A2], threads=4) == [per_dp(A2)] * 2


def test_cubic_window_schrijver_bregman():
    """3-regular 0-1 matrices: (4/3)^n <= per <= 6^(n/3) (Schrijver lower, Bregman upper bound)."""
    mats = W.config_n24() + [A for _, A in W.config_n60(4)]
    vals = native.hper_batch(mats, threads=8)
    for A, v in zip(mats, vals):
        n = A.shape[0]
        assert (4 / 3) ** n <= v <= 6 ** (n / 3)


def test_quartic_window():
    """4-regular 0-1 matrices: (27/16)^n <= per <= 24^(n/4) (Schrijver lower, Bregman upper bound)."""
    for s in range(3):
        A = W.random_quartic_matrix(24, s)
        v = per_dp(A)
        assert (27 / 16) ** 24 <= v <= 24 ** 6


def test_hper_dp_agree_on_cubic_n24_and_n40():
    mats = W.config_n24(range(4)) + [W.random_cubic_matrix(40, s) for s in range(2)]
    assert native.hper_batch(mats, threads=8) == [per_dp(A) for A in mats]
    assert per_hybrid(mats[0]) == per_dp(mats[0])


# --------------------------------------------------------------------------- KKLLL
def test_splitmix64_reference_outputs():
    """First outputs of SplitMix64 seeded with 0, as printed by its reference implementation."""
    assert [splitmix64(0, k) for k in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                   0x06C45D188009454F]


def test_kkl_exponents_are_uniform():
    counts = np.zeros(3)
    for t in range(40):
        for i in range(10):
            for j in range(10):
                counts[kkl_exponent(7, 3, t, i, j)] += 1
    expected = counts.sum() / 3
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 13.8  # 99.9% quantile of chi-square with 2 degrees of freedom


@pytest.mark.parametrize("seed", range(6))
def test_kkl_unbiased_by_exhaustive_enumeration(seed):
    """The KKLLL theorem E[|det B|^2] = per(A), checked exactly: average over all 3^nnz exponents."""
    rng = np.random.default_rng(seed)
    n = 3
    A = (rng.random((n, n)) < 0.7).astype(int)
    pos = list(zip(*np.nonzero(A)))
    if len(pos) > 8:
        pos = pos[:8]
        A = np.zeros((n, n), int)
        for i, j in pos:
            A[i, j] = 1
    total = 0.0
    for us in itertools.product(range(3), repeat=len(pos)):
        u = np.zeros((n, n), int)
        for (i, j), e in zip(pos, us):
            u[i, j] = e
        total += kkl_trial(A, u)
    assert abs(total / 3 ** len(pos) - per_brute(A)) < 1e-9


def test_kkl_single_permutation_gives_one():
    p = np.random.default_rng(0).permutation(9)
    A = np.zeros((9, 9), int)
    A[np.arange(9), p] = 1
    for t in range(5):
        u = np.random.default_rng(t).integers(0, 3, size=(9, 9))
        assert abs(kkl_trial(A, u) - 1.0) < 1e-12


# --------------------------------------------------------------------------- jobs of PH (expand_leaves)
def _line_counts(job):
    J = np.asarray(job)
    return np.count_nonzero(J, axis=1), np.count_nonzero(J, axis=0)


@pytest.mark.parametrize("seed", range(16))
def test_expand_leaves_sum_to_permanent_random_integer(seed):
    """Step 4 of Algorithm PH: the pre-expansion's jobs sum to per(A), checked against the
    definition (eq. 1) on non-symmetric integer matrices, at several cut-off orders."""
    n = 5 + seed % 5
    A = rand_int(n, 3000 + seed, hi=6, density=0.5)
    want = per_brute(A)
    for m_cut in range(1, n + 1):
        jobs = P.expand_leaves(A, m_cut)
        assert sum(per_brute(j) for j in jobs) == want
        for j in jobs:
            rows, cols = _line_counts(j)
            assert len(j) <= max(m_cut, 2)          # the size stop (no s >= 5 line here)
            assert rows.min() > 0 and cols.min() > 0   # a node with an empty line is dropped


@pytest.mark.parametrize("m_cut", [4, 8, 12, 16, 20])
def test_expand_leaves_sum_to_permanent_cubic_n24(m_cut):
    """The same identity on cubic graphs of 24 vertices against the independent frontier DP."""
    for s in range(2):
        A = W.random_cubic_matrix(24, s)
        jobs = P.expand_leaves(A, m_cut)
        assert all(len(j) == m_cut for j in jobs)   # cubic: every line has <= 4 nonzeros above m_cut
        assert sum(per_dp(j) for j in jobs) == per_dp(A)


def test_expand_leaves_s_leaf_branch_and_forced_split():
    """H_per's R-NW condition (every line has >= s_leaf nonzeros) makes a node a job while its
    order is <= m_cap; above m_cap such a node is split anyway. Dense 8 x 8 integer matrix:
    every line holds 8 nonzeros."""
    rng = np.random.default_rng(11)
    A = rng.integers(1, 4, size=(8, 8))
    want = per_brute(A)
    # s >= 5 and order <= m_cap: the root itself is the only job
    jobs = P.expand_leaves(A, m_cut=2, s_leaf=5, m_cap=8)
    assert len(jobs) == 1 and np.array_equal(np.asarray(jobs[0]), A)
    # m_cap = 7: the root is split (a full row gives ceil(8/2) = 4 children of order 7), each
    # child still has every line >= 5 nonzeros and order 7 <= m_cap, so each is a job
    jobs = P.expand_leaves(A, m_cut=2, s_leaf=5, m_cap=7)
    assert [len(j) for j in jobs] == [7, 7, 7, 7]
    assert sum(per_brute(j) for j in jobs) == want
    # m_cap = 5: forced splits continue down to order 5
    jobs = P.expand_leaves(A, m_cut=2, s_leaf=5, m_cap=5)
    assert jobs and all(len(j) == 5 for j in jobs)
    assert all(_line_counts(j)[0].min() >= 5 for j in jobs)
    assert sum(per_brute(j) for j in jobs) == want
    # s_leaf above every line count: plain size stop
    jobs = P.expand_leaves(A, m_cut=6, s_leaf=9, m_cap=8)
    assert all(len(j) == 6 for j in jobs) and sum(per_brute(j) for j in jobs) == want


def test_expand_leaves_drops_zero_nodes_and_limit():
    """A matrix with a zero column has no jobs (per = 0); ``limit`` keeps a prefix of the sequence."""
    A = rand_int(7, 77, hi=3, density=0.8)
    A[:, 3] = 0
    assert P.expand_leaves(A, 3) == []
    B = W.random_cubic_matrix(24, 5)
    full = P.expand_leaves(B, 16)
    assert P.expand_leaves(B, 16, limit=7) == full[:7]


# --------------------------------------------------------------------------- KKLLL key
def test_kkl_key_is_zero_for_permutation_patterns():
    """Every trial of a permutation (or of a block-diagonal of 1 x 1 blocks after any row and
    column shuffle) has |det B|^2 = 1, so the log-mean key is exactly 0."""
    from oracle import kkl_key
    rng = np.random.default_rng(5)
    for n in (1, 4, 9, 16):
        p = rng.permutation(n)
        A = np.zeros((n, n), int)
        A[np.arange(n), p] = 3   # the pattern is what counts, not the value
        for job in (0, 17):
            assert abs(kkl_key(A, 24, seed=9, job=job)) < 1e-12


@pytest.mark.parametrize("k,per,hadamard", [(2, 2, 4), (3, 6, 27)])
def test_kkl_key_mean_within_clt_interval(k, per, hadamard):
    """exp(key) is the mean of T independent trials of X = |det B|^2 with E[X] = per(J_k) = k!.
    Each X lies in [0, k^k] (Hadamard's inequality on rows of modulus-one entries), so its
    variance is at most (k^k)^2 / 4 (Popoviciu): the mean lies within 5 standard errors of k!."""
    from oracle import kkl_key
    T = 3000
    mean = math.exp(kkl_key(np.ones((k, k), int), T, seed=3, job=k))
    se = math.sqrt(hadamard ** 2 / 4 / T)
    assert abs(mean - per) < 5 * se
    # J_2 in closed form: X = |w^a w^d - w^b w^c|^2 is 0 (prob 1/3) or 3 (prob 2/3): variance 2
    if k == 2:
        assert abs(mean - 2) < 5 * math.sqrt(2 / T)


def test_kkl_key_is_log_of_the_trial_mean():
    """The key aggregates trials as the log of their arithmetic mean (not a mean of logs): for a
    matrix whose trials are 0 or 3 the mean of logs would be -inf."""
    from oracle import kkl_key
    from oracle.kkl import kkl_exponents
    A = np.ones((2, 2), int)
    xs = [kkl_trial(A, kkl_exponents(A, 4, 2, t)) for t in range(12)]
    assert set(round(x, 9) for x in xs) <= {0.0, 3.0} and 0.0 in [round(x, 9) for x in xs]
    assert abs(kkl_key(A, 12, 4, 2) - math.log(sum(xs) / 12)) < 1e-12
    Z = np.zeros((3, 3), int)
    Z[0, 0] = Z[1, 1] = 1   # a zero row: every trial is 0
    assert kkl_key(Z, 5, 1, 0) == float("-inf")
