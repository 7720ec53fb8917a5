"""The permanental polynomial per(xI - A): the oracle's two routes against each other and
against closed forms, then the library (GPU) against the oracle."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import per_brute
from oracle.permanent import per_dp
from oracle.polynomial import interpolate, perpoly_interpolate, perpoly_subsets

C60_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c60_permanental_polynomial.json")


def c60_coefficients() -> list[int]:
    with open(C60_GOLDEN) as fh:
        return [int(v) for v in json.load(fh)["coefficients"]]


def cycles(adj, k: int) -> int:
    """Number of cycles of length k >= 3 in a simple graph (each found from its least vertex,
    once per direction)."""
    count = 0

    def walk(start, v, depth, seen):
        nonlocal count
        for w in adj[v]:
            if w == start and depth == k:
                count += 1
            elif w > start and w not in seen and depth < k:
                seen.add(w)
                walk(start, w, depth + 1, seen)
                seen.discard(w)

    for s in range(len(adj)):
        walk(s, s, 1, {s})
    return count // 2


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


def test_c60_stored_polynomial_closed_forms():
    """The stored coefficients of per(xI - A) for C60 against graph counts. For a 0-1 symmetric
    A with zero diagonal, a_(n-s) (the sum of the permanents of the principal sub-matrices of order
    s) counts the covers of s vertices by disjoint edges and cycles, a cycle of length >= 3 counting
    twice (its two directions). With no triangles or 4-cycles: c_n = 1, c_(n-1) = 0,
    c_(n-2) = |E|, c_(n-3) = 0, c_(n-4) = pairs of disjoint edges, c_(n-5) = -2 (5-cycles),
    c_(n-6) = triples of disjoint edges + 2 (6-cycles); c_0 = per(A) by the oracle's H_per."""
    from oracle import native
    c = c60_coefficients()
    adj = W.read_appendix_adjacency("c60")
    n = len(adj)
    assert len(c) == n + 1 == 61
    E = [(i, j) for i in range(n) for j in adj[i] if i < j]
    assert cycles(adj, 3) == 0 and cycles(adj, 4) == 0
    c5, c6 = cycles(adj, 5), cycles(adj, 6)
    assert (c5, c6) == (12, 20)   # the pentagons and hexagons of the fullerene
    m2 = sum(1 for a, b in itertools.combinations(E, 2) if len({*a, *b}) == 4)
    m3 = sum(1 for a, b, d in itertools.combinations(E, 3) if len({*a, *b, *d}) == 6)
    assert c[60] == 1 and c[59] == 0 and c[58] == len(E) == 90 and c[57] == 0
    assert c[56] == m2 and c[55] == -2 * c5 and c[54] == m3 + 2 * c6
    assert c[0] == native.hper_batch([W.adjacency_matrix(adj)], threads=4)[0]
    # signs alternate with n - k: every a_k is a sum of non-negative permanents
    assert all(v == 0 or (v < 0) == bool((n - k) & 1) for k, v in enumerate(c))


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
        # orders above 64 whose values pass the exact rings' 2^180 are refused
        with pytest.raises(hperm.HpermError) as e:
            c.permanental_polynomial(W.random_cubic_matrix(70, 0))
        assert e.value.status == -2
    finally:
        c.close()


@pytest.mark.gpu
def test_modular_polynomial_matches_oracle(hperm):
    """Orders 23..64 past 2^180: the polynomial modulo primes below 2^18 and the Chinese
    remainder theorem on its coefficients. A cubic graph on 40 vertices (per(40I + A) about
    2^217; the 0-1 bound on the coefficients) and a weighted cubic graph on 36 vertices with
    diagonal entries (the row-sum bound) against the oracle's frontier DP and interpolation."""
    rng = np.random.default_rng(40)
    G = W.random_cubic_matrix(40, 0)
    H = (W.random_cubic_matrix(36, 2).astype(np.int64) * rng.integers(1, 8, (36, 36))
         + np.diag(rng.integers(0, 3, 36))).astype(np.uint32)
    c = hperm.Context()
    try:
        for A in (G, H):
            got = c.permanental_polynomial(A)
            assert got == perpoly_interpolate(A.astype(np.int64)), A.shape
    finally:
        c.close()


@pytest.mark.gpu
def test_mod_batch_equals_exact_residues(hperm):
    """per(A) mod p on the device path against exact values reduced mod p: the n = 60 cubic
    batch (oracle's stored values) and weighted cubic graphs with entries beyond p (frontier DP),
    for the largest prime below 2^18, 65537 and small primes."""
    import json as _json
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")
    with open(gold) as fh:
        stored = _json.load(fh)
    mats, exact = [], []
    for name, A in W.config_n60():
        mats.append(A)
        exact.append(int(stored[name]))
    rng = np.random.default_rng(23)
    for n, seed in ((24, 1), (30, 3), (44, 5)):
        A = (W.random_cubic_matrix(n, seed).astype(np.int64) * rng.integers(1, 1 << 20, (n, n))).astype(np.uint32)
        mats.append(A)
        exact.append(per_dp(A.astype(np.int64).tolist()))
    c = hperm.Context()
    try:
        for p in (262139, 65537, 7, 3):
            got = c.permanent_mod_batch(mats, p)
            assert got == [v % p for v in exact], p
        c.set_opts(split_order=14)   # leaves of order 14: the residue walk with 16 rows
        assert c.permanent_mod_batch(mats, 262139) == [v % 262139 for v in exact]
        c.set_opts(split_order=12)
        with pytest.raises(hperm.HpermError):
            c.permanent_mod_batch(mats[:1], 65535)   # not prime
        with pytest.raises(hperm.HpermError):
            c.permanent_mod_batch([W.random_cubic_matrix(20, 0)], 65537)   # order within the expansion
    finally:
        c.close()


@pytest.mark.gpu
def test_c60_evaluations_equal_stored_polynomial(hperm):
    """C60 at full size on sampled points: per(xI + A) mod p on the device path equals
    sum_k |c_k| x^k mod p from the stored coefficients (x = 0, 1 and 60; per(60I + A) is about
    2^358). Each point with x > 0 is a tree of about 2e9 leaves (every row gains the diagonal),
    so the whole polynomial (61 points, 6 primes) is a long run, not a test."""
    import time
    coeffs = c60_coefficients()
    A = W.adjacency_matrix(W.read_appendix_adjacency("c60")).astype(np.uint32)
    xs = (0, 1, 60)
    mats = [A + np.uint32(x) * np.eye(60, dtype=np.uint32) for x in xs]
    p = 262139
    c = hperm.Context()
    try:
        t0 = time.perf_counter()
        got = c.permanent_mod_batch(mats, p)
        print(f"C60 per(xI + A) mod {p} at x = {xs}: {time.perf_counter() - t0:.2f} s", flush=True)
        assert got == [sum(abs(v) * x ** k for k, v in enumerate(coeffs)) % p for x in xs]
    finally:
        c.close()


def c60_primes() -> list[int]:
    """The six largest primes below 2^18 (the residue route's primes for C60: five cover the
    coefficient bound max_k C(60, k) 6^(k/3) = 2^86.4 with two bits to spare, the sixth checks)."""
    out, q = [], (1 << 18) - 1
    while len(out) < 6:
        if all(q % d for d in range(2, int(q ** 0.5) + 1)):
            out.append(q)
        q -= 2
    return out


def test_polynomial_from_residues(hostlib):
    """The residue host step on C60's stored polynomial: its values at x = 0..60 reduced modulo
    the six primes give back the coefficients with alternating signs; a wrong residue, or too
    few primes for the coefficients, is caught by the check prime."""
    c = c60_coefficients()
    a = [abs(v) for v in c]
    primes = c60_primes()
    res = [[sum(ak * x ** k for k, ak in enumerate(a)) % p for x in range(61)] for p in primes]
    assert hostlib.polynomial_from_residues(primes, res, alternate=True) == c
    assert hostlib.polynomial_from_residues(primes, res) == a
    bad = [row[:] for row in res]
    bad[2][17] = (bad[2][17] + 1) % primes[2]
    with pytest.raises(hostlib.HpermError):
        hostlib.polynomial_from_residues(primes, bad)
    with pytest.raises(hostlib.HpermError):   # two primes: 36 bits for 50-bit coefficients
        hostlib.polynomial_from_residues(primes[:2] + primes[-1:], [res[0], res[1], res[-1]])
    with pytest.raises(hostlib.HpermError):   # not a prime
        hostlib.polynomial_from_residues([65535, 65537], [[0] * 61, [0] * 61])
