"""per(A) beyond the exact paths' range, evaluated by residues (the device path modulo primes,
the Chinese remainder theorem), against the oracle's frontier DP: through the batch call (alone
and mixed with problems of the exact paths) and through the serving loop."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.permanent import per_dp

RES = 1 << 3   # arith_mask bit of the residue ring


def big_entry_cubic(n: int, seed: int) -> np.ndarray:
    """A cubic 0-1 matrix with two entries raised to 2^21 - 1: a proven bound below 2^102 (the
    exact device path takes it), while the expansion's merges can carry an entry past 2^22."""
    A = W.random_cubic_matrix(n, seed).astype(np.uint32)
    nz = np.argwhere(A > 0)
    rng = np.random.default_rng(seed)
    for i, j in nz[rng.choice(len(nz), 2, replace=False)]:
        A[i, j] = (1 << 21) - 1
    return A


def out_of_range_cases():
    rng = np.random.default_rng(7)
    return [
        # expanded entries pass 2^22 on the host path (bounds 2^137, 2^163)
        ("union48", W.permutation_union_matrix(48, 3, 48)),
        ("union56", W.permutation_union_matrix(56, 3, 56)),
        # the bound (2^425) passes the host path's 2^180
        ("cubic40_w2^10", (W.random_cubic_matrix(40, 11).astype(np.int64)
                           * rng.integers(1, 1 << 10, (40, 40))).astype(np.uint32)),
    ]


def log2_bound(A) -> float:
    A = np.asarray(A, dtype=np.float64)
    return min(sum(math.log2(x) for x in A.sum(1)), sum(math.log2(x) for x in A.sum(0)))


@pytest.mark.gpu
def test_out_of_range_problems_by_residues(hperm):
    cases = out_of_range_cases()
    want = [per_dp(A.astype(np.int64).tolist()) for _, A in cases]
    c = hperm.Context()
    try:
        for (name, A), v in zip(cases, want):
            print("residues", name, f"bound 2^{log2_bound(A):.0f}", flush=True)
            got, st = c.permanent_batch([A], with_stats=True)
            assert got == [v], name
            assert st[0]["arith_mask"] == RES, name
            launches = c.last_launches()
            assert launches[-1]["variant"] == 5 and launches[-1]["ring"] == 2
            assert launches[-1]["row_updates"] >= 3   # primes: K covering the bound, and a check
        # one batch: the three, an exact device-path problem and a small host-path problem
        small = W.random_cubic_matrix(16, 1)
        c60 = W.adjacency_matrix(W.truncated_icosahedron())
        mats = [A for _, A in cases] + [c60, small]
        exact = want + [per_dp(c60.astype(np.int64).tolist()), per_dp(small.astype(np.int64).tolist())]
        got, st = c.permanent_batch(mats, with_stats=True)
        assert got == exact
        assert [s["arith_mask"] == RES for s in st] == [True, True, True, False, False]
    finally:
        c.close()


@pytest.mark.gpu
def test_device_path_overflow_falls_back_to_residues(hperm):
    """Problems the exact device path takes by their bound whose expansion carries an entry past
    2^22: the group is evaluated again by residues."""
    mats = [big_entry_cubic(30, s) for s in (3, 4)]
    for A in mats:
        assert log2_bound(A) < 102
    want = [per_dp(A.astype(np.int64).tolist()) for A in mats]
    c = hperm.Context()
    try:
        got, st = c.permanent_batch(mats, with_stats=True)
        print("device overflow arith", [s["arith_mask"] for s in st], flush=True)
        assert got == want
        assert all(s["arith_mask"] == RES for s in st)
    finally:
        c.close()


@pytest.mark.gpu
def test_serving_out_of_range_requests(hperm):
    """The serving loop routes out-of-range requests to the device lane's residue evaluation,
    interleaved with ordinary requests."""
    cases = out_of_range_cases()[:1] + out_of_range_cases()[2:]
    small = [W.random_cubic_matrix(20, s) for s in range(3)]
    mats = [cases[0][1], small[0], cases[1][1], small[1], small[2]]
    want = [per_dp(A.astype(np.int64).tolist()) for A in mats]
    c = hperm.Context()
    try:
        c.serve_start()
        tickets = [c.submit(A) for A in mats]
        assert all(t is not None for t in tickets)
        out = [c.wait(t, 120.0) for t in tickets]
        c.serve_stop()
        assert [v for v, _ in out] == want
        assert [s["arith_mask"] == RES for _, s in out] == [True, False, True, False, False]
    finally:
        c.close()


@pytest.mark.gpu
def test_largest_order_by_residues(hperm):
    """Order 128 (the largest input): per(2I + P) = 2^128 + 1 for the cyclic shift P, whose bound
    3^128 = 2^203 passes the host path's 2^180, by residues (primes below 2^17, so that 128 (p - 1)
    < 2^24); a bound beyond 2^500 (17^128) is refused."""
    eye = np.eye(128, dtype=np.uint32)
    P = np.roll(eye, 1, axis=1)
    c = hperm.Context()
    try:
        got, st = c.permanent_batch([2 * eye + P], with_stats=True)
        assert got == [2 ** 128 + 1]
        assert st[0]["arith_mask"] == RES
        with pytest.raises(hperm.HpermError) as e:
            c.permanent(16 * eye + P)
        assert e.value.status == -2
    finally:
        c.close()
