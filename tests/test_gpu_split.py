"""GPU parity of the device continuation of Algorithm H_per (split_order): each job is split
on the device by expansion (2) down to the target order and its leaves evaluated by R-NW in
the same kernel. Per-job values are compared bit-exact with the oracle's permanent of the job's
sub-matrix; the traversal (number of leaves and their subset-terms) with the oracle's own
H_per expansion of the same sub-matrix (``expand_leaves``, the same splitting rule)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import expand_leaves, native

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "oracle_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def job_mats(J):
    return [J.matrix(k).astype(np.int64).tolist() for k in range(J.info()[0])]


def oracle_traversal(mats, t):
    """(leaves, leaf subset-terms) of the oracle's H_per expansion of the jobs of order > t."""
    leaves = terms = 0
    for B in mats:
        if len(B) <= t:
            continue
        for leaf in expand_leaves(B, t, 5, 40):
            leaves += 1
            terms += 1 << (len(leaf) - 1)
    return leaves, terms


def split_launch(ctx):
    ls = [l for l in ctx.last_launches() if l["variant"] == 3]
    assert len(ls) == 1
    return ls[0]


@pytest.fixture(scope="module")
def ctx(hperm):
    c = hperm.Context()
    yield c
    c.close()


@pytest.mark.parametrize("t", [7, 10, 12, 13, 15])
def test_split_jobs_match_oracle(hperm, ctx, t):
    """Cubic graphs on 26 vertices expanded to jobs of order <= 16 on the host, continued on the
    device to order t: every job's value and the totals equal the oracle's, and the device
    reaches exactly the oracle's leaves (t = 13 and 15: leaves walked with 16 rows, in blocks of
    four steps where two sparse columns are disjoint)."""
    for seed in range(3):
        A = W.random_cubic_matrix(26, seed)
        say("split parity", t, "seed", seed)
        ctx.set_opts(m_cut=16, split_order=t)
        try:
            J = ctx.expand([A])
            totals, per_job, _ = ctx.run(J, "natural", True, per_job=True)
            st = split_launch(ctx)
        finally:
            ctx.set_opts(m_cut=20, split_order=0)
        mats = job_mats(J)
        assert per_job == native.ryser_batch(mats, threads=8)
        assert totals == [sum(per_job)]
        assert st["n_jobs"] == sum(1 for B in mats if len(B) > t)
        assert st["split_stops"] == 0
        assert (st["leaves"], st["leaf_terms"]) == oracle_traversal(mats, t)


def test_split_n24_golden(hperm, ctx):
    """Ten cubic graphs on 24 vertices end to end with the default cut-off and split order 12."""
    mats = W.config_n24()
    say("split n24 golden")
    ctx.set_opts(split_order=12)
    try:
        got = ctx.permanent_batch(mats)
    finally:
        ctx.set_opts(split_order=0)
    assert got == [int(GOLDEN[f"cubic24_seed{s}"]) for s in range(10)]


def test_split_mixed_table(hperm, ctx):
    """A job table mixing jobs the device splits (mod 2^64, order 13..20), jobs too small to
    split, dense jobs that are leaves at their own order (every line >= 5 nonzeros: the 16- and
    20-row leaf walks) and jobs of wider rings: all values equal the oracle's."""
    mats = []
    for i, m in enumerate((5, 8, 12, 13, 15, 17, 19, 20)):
        mats.append(W.permutation_union_matrix(m, 3, 700 + i, 1, 3))
    for m in (13, 14):                            # all-ones: leaves at their own order
        mats.append(np.ones((m, m), np.uint32))
    for i, m in enumerate((16, 17, 18)):          # eight permutations: most lines >= 5 nonzeros
        mats.append(W.permutation_union_matrix(m, 8, 800 + i, 1, 1))
    mats.append(W.permutation_union_matrix(14, 3, 900, 20, 60))       # entries force a wider ring
    J = ctx.jobs_from_dense(mats)
    d = J.describe()
    say("split mixed", list(d["m"]), list(d["arith"]))
    ctx.set_opts(split_order=12)
    try:
        totals, per_job, _ = ctx.run(J, "natural", True, per_job=True)
        st = split_launch(ctx)
    finally:
        ctx.set_opts(split_order=0)
    stored = job_mats(J)
    assert per_job == native.ryser_batch(stored, threads=8)
    eligible = [B for B, a in zip(stored, d["arith"]) if a == 1 and 12 < len(B) <= 20]
    assert st["n_jobs"] == len(eligible)
    assert (st["leaves"], st["leaf_terms"]) == oracle_traversal(eligible, 12)
    assert max(len(x) for B in eligible for x in expand_leaves(B, 12, 5, 40)) > 16   # wide leaves ran
    assert max(d["arith"]) > 1


@pytest.mark.parametrize("order", ["natural", "estimate", "random", "exact_cost"])
def test_split_n60_bench_workload(hperm, ctx, order):
    """The benchmark workload (17 cubic graphs on 60 vertices, 324386 jobs of order 20)
    continued to order 12: totals equal the oracle's, and sampled jobs equal the oracle's
    permanent of their sub-matrices."""
    items = W.config_n60(16)
    say("split n60", order)
    J = ctx.expand([A for _, A in items])
    if order == "estimate":
        ctx.estimate(J, 32, 1)
    ctx.set_opts(split_order=12)
    try:
        totals, per_job, _ = ctx.run(J, order, True, per_job=(order == "natural"))
        st = split_launch(ctx)
    finally:
        ctx.set_opts(split_order=0)
    assert totals == [int(GOLDEN[name]) for name, _ in items]
    say("split n60 leaves", st["leaves"], "leaf terms", st["leaf_terms"], "ms", st["ms"],
        "stops", st["split_stops"])
    if per_job is not None:
        rng = np.random.default_rng(3)
        pick = sorted(rng.choice(len(per_job), 24, replace=False).tolist())
        mats = [J.matrix(k).astype(np.int64).tolist() for k in pick]
        assert [per_job[k] for k in pick] == native.ryser_batch(mats, threads=8)


def test_split_job_timing(hperm):
    """time_jobs = 1 with split_order: every split job gets positive work cycles; values
    unchanged."""
    c = hperm.Context({"time_jobs": 1, "split_order": 10})
    try:
        mats = [W.permutation_union_matrix(m, 3, 600 + m, 1, 2) for m in (14, 18, 20)]
        J = c.jobs_from_dense(mats)
        _, per_job, _ = c.run(J, "natural", True, per_job=True)
        assert per_job == native.ryser_batch(job_mats(J), threads=8)
        assert (J.cycles() > 0).all()
    finally:
        c.close()


def test_split_serving_and_arena(hperm):
    """The serving loop and a caller-owned device arena with split_order: served values and
    batch values equal the oracle's (mixed 3-regular, 4-regular and small-integer requests)."""
    reqs = [A for _, A in W.serving_requests(24, 11, 18, 32)]
    want = native.hper_batch(reqs, threads=8)
    say("split serving", len(reqs))
    c = hperm.Context({"m_cut": 16, "split_order": 10})
    try:
        c.serve_start(32, 64 << 20)
        tickets = [c.submit(A) for A in reqs]
        assert all(t is not None for t in tickets)
        got = [c.wait(t, 120.0)[0] for t in tickets]
        c.serve_stop()
        assert got == want
        c.set_arena(4096)
        got, seen = None, []
        for _ in range(8):   # each refusal reports what its allocation needed
            try:
                got = c.permanent_batch(reqs)
                break
            except hperm.HpermError as e:
                seen.append((e.status, str(e)[-60:], c.arena_required()))
                assert e.status == -4, seen
                c.set_arena(c.arena_required() * 2)
        say("arena attempts", seen)
        assert got == want, seen
    finally:
        c.close()


def test_split_extremes(hperm, ctx):
    """Target 19 (one split level below order 20), target 7 (the smallest), and job tables
    with nothing to split (no device H_per launch): values equal the oracle's."""
    mats = [W.permutation_union_matrix(20, 3, 30 + i, 1, 2) for i in range(4)]
    mats += [W.permutation_union_matrix(m, 3, 40 + m, 1, 2) for m in (8, 9, 11)]
    J = ctx.jobs_from_dense(mats)
    stored = job_mats(J)
    want = native.ryser_batch(stored, threads=8)
    eligible = lambda t: [B for B, a in zip(stored, J.describe()["arith"]) if a == 1 and t < len(B) <= 20]
    for t in (19, 7):
        say("split extreme", t)
        ctx.set_opts(split_order=t)
        try:
            _, per_job, _ = ctx.run(J, "natural", True, per_job=True)
            st = split_launch(ctx)
        finally:
            ctx.set_opts(split_order=0)
        assert per_job == want
        assert (st["leaves"], st["leaf_terms"]) == oracle_traversal(eligible(t), t)
    small = ctx.jobs_from_dense([W.permutation_union_matrix(m, 3, 50 + m, 1, 2) for m in (5, 9, 12)])
    ctx.set_opts(split_order=12)
    try:
        _, per_job, _ = ctx.run(small, "natural", True, per_job=True)
        assert not [l for l in ctx.last_launches() if l["variant"] == 3]
    finally:
        ctx.set_opts(split_order=0)
    assert per_job == native.ryser_batch(job_mats(small), threads=8)


def test_split_from_order_24(hperm, ctx):
    """Jobs of order 21..24 split on the device: ten cubic graphs on 24 vertices, each a single
    job (m_cut 24), and the benchmark's graphs expanded by the host only down to order 24;
    per-job values and the traversal against the oracle's, totals against the stored values."""
    mats = W.config_n24()
    say("split from 24: n24 single jobs")
    ctx.set_opts(m_cut=24, split_order=12)
    try:
        J = ctx.expand(mats)
        totals, per_job, _ = ctx.run(J, "natural", True, per_job=True)
        st = split_launch(ctx)
    finally:
        ctx.set_opts(m_cut=20, split_order=0)
    stored = job_mats(J)
    assert sorted(len(B) for B in stored)[-1] == 24
    assert totals == [int(GOLDEN[f"cubic24_seed{s}"]) for s in range(10)]
    assert per_job == native.ryser_batch(stored, threads=8)
    eligible = [B for B, a in zip(stored, J.describe()["arith"]) if a == 1 and 12 < len(B) <= 24]
    assert st["n_jobs"] == len(eligible)
    assert (st["leaves"], st["leaf_terms"]) == oracle_traversal(eligible, 12)
    mixed = [W.permutation_union_matrix(m, 3, 70 + m, 1, 1) for m in (21, 22, 23, 24)]   # 0-1: mod 2^64
    J2 = ctx.jobs_from_dense(mixed)
    ctx.set_opts(split_order=14)
    try:
        _, pj2, _ = ctx.run(J2, "natural", True, per_job=True)
        st2 = split_launch(ctx)
    finally:
        ctx.set_opts(split_order=0)
    stored2 = job_mats(J2)
    assert pj2 == native.ryser_batch(stored2, threads=8)
    el2 = [B for B, a in zip(stored2, J2.describe()["arith"]) if a == 1 and 14 < len(B) <= 24]
    assert (st2["leaves"], st2["leaf_terms"]) == oracle_traversal(el2, 14)
    items = W.config_n60(16)
    say("split from 24: n60")
    ctx.set_opts(m_cut=24, split_order=12)
    try:
        got = ctx.permanent_batch([A for _, A in items])
    finally:
        ctx.set_opts(m_cut=20, split_order=0)
    assert got == [int(GOLDEN[name]) for name, _ in items]


def refusing_job(hperm, m, seed):
    """A job of order m whose first H_per split must be refused. The base pattern is a 0-1
    cycle (row r on columns r and r+1 mod m) with row 0 cut to the single entry 2^11 at
    column 0 and one extra 1 at (2, 1), rows and columns permuted by the seed: that row is
    the unique sparsest line, and the odd entry's split scales the lowest zero column of
    its row (in the job's stored order) by 2^11. One more 2^11 is placed, by a seeded
    search, on an entry that the oracle's own first split of the stored job multiplies by
    the first: a child entry reaches 2^22, beyond the entry limit, so the device keeps the
    job whole (a leaf of order m); the bound keeps the job in the mod-2^64 ring."""
    from oracle.permanent import choose_line, e2_children
    rng = np.random.default_rng(seed)
    base = np.zeros((m, m), np.uint32)
    for r in range(1, m):
        base[r, r] = base[r, (r + 1) % m] = 1
    base[0, 0] = 1 << 11
    base[2, 1] = 1
    base = base[rng.permutation(m)][:, rng.permutation(m)]
    host = hperm.Context(host_only=True)
    try:
        cand = [tuple(x) for x in np.argwhere(base == 1)]
        for k in rng.permutation(len(cand)):
            A = base.copy()
            A[cand[k]] = 1 << 11
            J = host.jobs_from_dense([A])
            if J.describe()["arith"][0] != 1:
                continue
            B = J.matrix(0).astype(np.int64).tolist()
            kind, idx, _ = choose_line(B)
            if max(max(max(r) for r in C) for C in e2_children(B, kind, idx)) >= 1 << 22:
                return A
    finally:
        host.close()
    raise AssertionError(f"no refusing placement for m={m}, seed {seed}")


@pytest.mark.parametrize("t", [7, 12])
def test_split_refused_at_entry_limit(hperm, ctx, t):
    """Jobs whose first split would merge two entries 2^11 into 2^22 (beyond the entry limit
    of the device arithmetic): the device refuses the split and evaluates the job whole, at
    order 14 and 16 by the leaf walk and at order 18 and 20 by the deferred 20-row replay;
    every job value equals the oracle's permanent of the stored sub-matrix."""
    mats = [refusing_job(hperm, m, 50 + m) for m in (14, 16, 18, 20)]
    mats.append(W.permutation_union_matrix(18, 3, 61, 1, 2))    # an ordinary job beside them
    J = ctx.jobs_from_dense(mats)
    assert list(J.describe()["arith"]) == [1] * len(mats)
    stored = job_mats(J)
    say("split refused", t)
    ctx.set_opts(split_order=t)
    try:
        totals, per_job, _ = ctx.run(J, "natural", True, per_job=True)
        st = split_launch(ctx)
    finally:
        ctx.set_opts(split_order=0)
    say("split refused stats", {k: st[k] for k in ("leaves", "splits", "split_stops", "deferred")})
    assert per_job == native.ryser_batch(stored, threads=8)
    assert totals == per_job              # one problem per matrix
    assert st["split_stops"] >= 4         # one refusal at each refusing job's root
    assert st["deferred"] >= 2            # the order-18 and order-20 roots, kept whole
