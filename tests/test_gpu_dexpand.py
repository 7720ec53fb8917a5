"""GPU parity of the device expansion (option device_expand = T): the expansion tree of
Algorithm H_per is built level by level on the GPU down to jobs of order T, which the device
continuation of H_per finishes, with per-leaf normalisation and 128-bit sums. Compared with the
oracle: per(A) against the C H_per oracle, the stored oracle values and the paper's printed
C100 total; the jobs themselves (matrices, in tree order) against the oracle's own expansion
``expand_leaves`` and their values against the oracle's permanents of them."""
import json
import math
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import expand_leaves, native
from oracle.permanent import per_dp

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "oracle_values.json")))
C100_PER = 149364113290700   # the paper's appendix: the total of the 159 sub-permanents


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nonzero_lines(B) -> bool:
    B = np.asarray(B)
    return bool((B != 0).any(axis=1).all() and (B != 0).any(axis=0).all())


def oracle_jobs(A, T, limit=None):
    """The oracle's jobs of order T: expansion (2) with H_per's line rule above T (a line of
    five or more nonzeros is split too, as the device does above the job order)."""
    return expand_leaves(np.asarray(A, dtype=np.int64), T, 10 ** 9, 40, limit=limit)


def device_ctx(hperm, T, t=12, mib=1024):
    return hperm.Context({"split_order": t, "device_expand": T, "device_expand_mib": mib})


@pytest.mark.parametrize("T,t", [(16, 7), (20, 12), (24, 12), (24, 20)])
def test_device_expansion_small_problems(hperm, T, t):
    """Cubic graphs on 26..44 vertices and small-integer matrices: per(A) equals the C H_per
    oracle for several job orders T and target orders t."""
    mats = [W.random_cubic_matrix(n, s) for n, s in [(26, 0), (30, 1), (36, 2), (44, 3)]]
    mats += [W.permutation_union_matrix(28, 3, 11, 1, 4), W.permutation_union_matrix(34, 3, 12, 1, 3),
             W.random_quartic_matrix(30, 5)]
    want = native.hper_batch(mats, threads=8)
    say("dexpand small", T, t)
    c = device_ctx(hperm, T, t)
    try:
        got = c.permanent_batch(mats)
        dev = [l for l in c.last_launches() if l["variant"] == 4]
    finally:
        c.close()
    assert got == want
    big = [A.shape[0] for A in mats if A.shape[0] > T]
    assert len(dev) == len(set(big))                 # one expansion per order
    assert sum(l["reserved"] for l in dev) == len(big)


@pytest.mark.parametrize("kind", ["cubic", "integer"])
def test_device_jobs_equal_oracle_expansion(hperm, kind):
    """Every job of the device expansion, in tree order, equals the oracle's expansion of the
    same matrix (jobs with an empty line, which the oracle drops, have value 0), and every job
    value equals the oracle's permanent of that job."""
    A = W.random_cubic_matrix(36, 7) if kind == "cubic" else W.permutation_union_matrix(38, 3, 24, 1, 3)
    T = 16
    want_jobs = oracle_jobs(A, T)
    c = device_ctx(hperm, T)
    try:
        total, jobs, vals, _ = c.device_expand_sample(A, 4096)
    finally:
        c.close()
    assert total == native.hper_batch([A], threads=8)[0]
    kept = [(B, v) for B, v in zip(jobs, vals) if nonzero_lines(B)]
    assert all(v == 0 for B, v in zip(jobs, vals) if not nonzero_lines(B))
    say("dexpand jobs", kind, len(jobs), "kept", len(kept), "oracle", len(want_jobs))
    assert len(kept) == len(want_jobs)
    for (B, _), Bo in zip(kept, want_jobs):
        assert B.tolist() == [[int(x) for x in r] for r in Bo]
    assert [v for _, v in kept] == native.hper_batch([B for B, _ in kept], threads=8)
    assert sum(vals) == total


def test_device_expansion_n60_and_mixed_batch(hperm):
    """The benchmark graphs (17 cubic graphs on 60 vertices) against the stored oracle values,
    at two job orders, and a batch mixing problems below T (host path) with problems above."""
    items = W.config_n60(16)
    mats = [A for _, A in items]
    c = device_ctx(hperm, 22)
    try:
        for T in (20, 22):
            c.set_opts(device_expand=T)
            say("dexpand n60", T)
            assert c.permanent_batch(mats) == [int(GOLDEN[n]) for n, _ in items]
        c.set_opts(device_expand=24)   # the graphs on 24 vertices stay on the host path
        mixed = W.config_n24(range(3)) + mats[:2]
        got = c.permanent_batch(mixed)
        dev = [l for l in c.last_launches() if l["variant"] == 4]
    finally:
        c.close()
    assert got == [int(GOLDEN[f"cubic24_seed{s}"]) for s in range(3)] + [int(GOLDEN[n]) for n, _ in items[:2]]
    assert len(dev) == 1 and dev[0]["reserved"] == 2   # the two graphs on 60 vertices together


def test_device_expansion_n80_golden(hperm):
    """The batched configuration's eight cubic graphs on 80 vertices against the stored oracle
    values."""
    items = W.config_n80(8)
    say("dexpand n80")
    c = device_ctx(hperm, 22, mib=4096)
    try:
        got = c.permanent_batch([A for _, A in items])
    finally:
        c.close()
    assert got == [int(GOLDEN[n]) for n, _ in items]


def test_c100_equals_the_paper(hperm):
    """per(A(C100)) of the paper's appendix on the device path, equal to the paper's printed
    total, and the first jobs of the device's tree equal the oracle's expansion of C100 with
    the oracle's permanents as values."""
    A = W.adjacency_matrix(W.read_appendix_adjacency("c100"))
    T, K = 22, 48
    say("dexpand C100")
    c = device_ctx(hperm, T, mib=8192)
    try:
        total, jobs, vals, st = c.device_expand_sample(A, K)
    finally:
        c.close()
    say("C100", total, st)
    assert total == C100_PER
    kept = [(B, v) for B, v in zip(jobs, vals) if nonzero_lines(B)]
    want_jobs = oracle_jobs(A, T, limit=len(kept))
    assert [B.tolist() for B, _ in kept] == [[[int(x) for x in r] for r in Bo] for Bo in want_jobs]
    assert [v for _, v in kept] == native.hper_batch([B for B, _ in kept], threads=8)


@pytest.mark.parametrize("seed", [0, 1])
def test_random_cubic_100_first_jobs(hperm, seed):
    """Random cubic graphs on 100 vertices (the large single-problem configuration) at full
    size: the device's first jobs of order 22 equal the oracle's expansion and their values the
    oracle's permanents (the run stops once they are kept)."""
    A = W.random_cubic_matrix(100, seed)
    T, K = 22, 64
    c = device_ctx(hperm, T, mib=8192)
    try:
        total, jobs, vals, _ = c.device_expand_sample(A, K, stop_early=True)
    finally:
        c.close()
    assert total is None and len(jobs) == K
    kept = [(B, v) for B, v in zip(jobs, vals) if nonzero_lines(B)]
    say("dexpand n100 seed", seed, "kept", len(kept))
    want_jobs = oracle_jobs(A, T, limit=len(kept))
    assert [B.tolist() for B, _ in kept] == [[[int(x) for x in r] for r in Bo] for Bo in want_jobs]
    assert [v for _, v in kept] == native.hper_batch([B for B, _ in kept], threads=8)


def test_device_expansion_limits(hperm):
    """Options out of range are refused; a problem at or below T, with a bound beyond 2^102 or
    with a zero column takes the host path; merged entries reaching 2^22 in the device
    expansion leave the exact rings and are evaluated by residues."""
    with pytest.raises(hperm.HpermError):
        hperm.Context({"split_order": 12, "device_expand": 25})
    for opts in ({"split_order": 12, "device_expand": 12}, {"split_order": 0, "device_expand": 20}):
        off = hperm.Context(opts)   # not in effect: the host path
        try:
            A = W.random_cubic_matrix(30, 2)
            assert off.permanent(A) == native.hper_batch([A])[0]
            assert not [l for l in off.last_launches() if l["variant"] == 4]
        finally:
            off.close()
    c = device_ctx(hperm, 20)
    try:
        small = W.random_cubic_matrix(20, 3)
        dense = np.ones((22, 22), np.uint32)           # bound log2 22! = 69.9: device path
        wide = np.ones((30, 30), np.uint32)            # bound log2 30! = 107.7: host path
        z = W.random_cubic_matrix(30, 4).copy()
        z[:, 5] = 0
        got = c.permanent_batch([small, dense, wide, z])
        kinds = [l["variant"] for l in c.last_launches()]
        assert got == [native.hper_batch([small])[0], math.factorial(22), math.factorial(30), 0]
        assert kinds.count(4) == 1
        # column 0 holds 2^21 in every row (column-sum bound 2^55): the first split merges it
        # into 2^22, past the exact rings' entry limit; the group is evaluated again by residues
        # (exact, never a wrong value)
        big = np.zeros((30, 30), np.uint32)
        big[:, 0] = 1 << 21
        for i in range(1, 30):
            big[i, i] = 1
        for i in range(29):
            big[i, i + 1] = 1
        got, st = c.permanent_batch([big], with_stats=True)
        assert got == [per_dp(big.astype(np.int64).tolist())]
        assert st[0]["arith_mask"] == 1 << 3
        assert [l["variant"] for l in c.last_launches()][-1] == 5
    finally:
        c.close()
