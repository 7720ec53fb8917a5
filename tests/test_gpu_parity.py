"""GPU parity: the HIP path against the CPU oracle, bit-exact (integers), through the C ABI.

Inputs come from the seeded generators in ``workloads``; expected values come from the
oracle (computed here, or stored in tests/golden/oracle_values.json by
tests/golden/make_golden.py, which calls only the oracle).
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import expand_leaves, kkl_key, native, per_brute, per_dp, per_ryser

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "oracle_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def leaf_like(m, seed, k=4, hi=8):
    """Job-like m x m matrix: the union of k random permutations, values U{1..hi} (per >= 1)."""
    return W.permutation_union_matrix(m, k, seed, 1, hi)


@pytest.fixture(scope="module")
def ctx(hperm):
    c = hperm.Context({"split_order": 0})   # these tests cover the R-NW kernels
    yield c
    c.close()


# ------------------------------------------------------------------ R-NW on given jobs
SIZES = [1, 2, 3, 5, 7, 8, 9, 12, 13, 16, 17, 19, 20]


@pytest.mark.parametrize("arith", ["auto", "w128", "res"])
@pytest.mark.parametrize("persistent", [True, False])
def test_jobs_random_integer(hperm, ctx, arith, persistent):
    mats = [leaf_like(m, 100 + i, k=3 + i % 4) for i, m in enumerate(SIZES)]
    want = native.ryser_batch(mats, threads=8)
    say("jobs_random_integer", arith, persistent, SIZES)
    ctx.set_opts(arith=arith)
    try:
        J = ctx.jobs_from_dense(mats)
        ctx.estimate(J, 8, 3)
        totals, per_job, _ = ctx.run(J, "estimate", persistent, per_job=True)
    finally:
        ctx.set_opts(arith="auto")
    assert per_job == want
    assert totals == want


@pytest.mark.parametrize("chunk", [1, 3, 6, 9])
def test_chunk_size_does_not_change_values(hperm, ctx, chunk):
    mats = [leaf_like(m, 7 + m) for m in (11, 15, 18)]
    want = native.ryser_batch(mats, threads=4)
    say("chunk", chunk)
    ctx.set_opts(chunk_log2=chunk)
    try:
        totals, per_job, _ = ctx.run(ctx.jobs_from_dense(mats), "natural", True, per_job=True)
    finally:
        ctx.set_opts(chunk_log2=0)
    assert per_job == want


@pytest.mark.parametrize("k", [1, 2, 6, 12, 16, 20, 22, 24])
def test_all_ones_is_factorial(hperm, ctx, k):
    """per(J_k) = k!: J_20 and J_24 need the 128-bit ring (bound + k bits of doubling)."""
    say("J", k)
    totals, _, res = ctx.run(ctx.jobs_from_dense([np.ones((k, k))]), "natural", True)
    assert totals == [math.factorial(k)]


def test_residue_ring_j30(hperm, ctx):
    """J_30: 30! ~ 2^107.7 plus 30 bits of doubling exceeds 128 bits: three residues + CRT."""
    say("J30 residues")
    J = ctx.jobs_from_dense([np.ones((30, 30))])
    assert list(J.describe()["arith"]) == [hperm.ARITH_RES]
    totals, _, _ = ctx.run(J, "natural", True)
    assert totals == [math.factorial(30)]


def test_scaled_all_ones(hperm, ctx):
    """per(c J_k) = c^k k!."""
    say("scaled J")
    mats = [np.full((9, 9), 7), np.full((14, 14), 3), np.full((17, 17), 2)]
    totals, _, _ = ctx.run(ctx.jobs_from_dense(mats), "natural", True)
    assert totals == [7 ** 9 * math.factorial(9), 3 ** 14 * math.factorial(14), 2 ** 17 * math.factorial(17)]


def test_job_orders_rows_32_to_40(hperm, ctx):
    """Jobs of order 33..36 use the second register array for rows 32 and up."""
    say("orders 33..36")
    mats = [np.eye(m, dtype=np.uint32) + np.roll(np.eye(m, dtype=np.uint32), 1, axis=1) for m in (33, 36)]
    # per(I + P) for the cyclic shift P is 2 (two permutations)
    totals, _, _ = ctx.run(ctx.jobs_from_dense(mats), "natural", True)
    assert totals == [2, 2]


def test_four_step_walks_every_order_bucket(hperm, ctx):
    """Sparse 0-1 jobs of orders 12..40 in the 64-bit ring whose first Gray columns take the
    four-step walks' shapes (column 0 on two or three rows, column 1 on rows disjoint from
    them): cubic graphs (three-row shape) and unions of two or three permutations (mostly the
    two-row shape), one or more per order bucket, job by job against the oracle's DP."""
    mats = ([W.random_cubic_matrix(n, 40 + n) for n in (12, 18, 22, 28, 32)]
            + [W.permutation_union_matrix(n, 3, 60 + n, 1, 1) for n in (16, 20, 24, 30, 33)]
            + [W.permutation_union_matrix(n, 2, 60 + n, 1, 1) for n in (22, 37, 40)])
    want = [per_dp(A.astype(np.int64).tolist()) for A in mats]
    say("four-step walks, orders", [A.shape[0] for A in mats])
    J = ctx.jobs_from_dense(mats)
    assert set(J.describe()["arith"]) == {hperm.ARITH_W64}
    totals, per_job, _ = ctx.run(J, "natural", True, per_job=True)
    launches = {(L["bucket"], L["variant"]) for L in ctx.last_launches()}
    assert per_job == want
    assert totals == want
    assert {(b, 7) for b in (0, 2, 3)} <= launches and {(b, 6) for b in (0, 2, 3, 4)} <= launches


# ------------------------------------------------------------------ expansion + R-NW
@pytest.mark.parametrize("m_cut", [10, 14])
def test_leaf_values_match_oracle_leaves(hperm, ctx, m_cut):
    """Job-by-job: the GPU value of each job equals the oracle's permanent of the oracle's own
    job in the same position of the depth-first expansion (both follow the same rule)."""
    A = W.random_cubic_matrix(24, 5)
    say("leaf parity", m_cut)
    ctx.set_opts(m_cut=m_cut)
    try:
        J = ctx.expand([A])
        ctx.estimate(J, 16, 1)
        totals, per_job, _ = ctx.run(J, "estimate", True, per_job=True)
    finally:
        ctx.set_opts(m_cut=20)
    leaves = expand_leaves(A, m_cut)
    assert per_job == native.ryser_batch(leaves, threads=8)
    assert totals == [int(GOLDEN["cubic24_seed5"])]


def test_n24_configs_end_to_end(hperm, ctx):
    mats = W.config_n24()
    say("n24 end to end")
    for m_cut in (12, 20):
        ctx.set_opts(m_cut=m_cut)
        got = ctx.permanent_batch(mats)
        assert got == [int(GOLDEN[f"cubic24_seed{s}"]) for s in range(10)]
    ctx.set_opts(m_cut=20)


def test_n60_configs_end_to_end(hperm, ctx):
    """The benchmark workload at full size: truncated icosahedron + 16 random cubic girth>=5."""
    items = W.config_n60(16)
    say("n60 end to end (bench configuration)")
    got, stats = ctx.permanent_batch([A for _, A in items], with_stats=True)
    assert got == [int(GOLDEN[name]) for name, _ in items]
    say("n60 jobs", sum(s["n_jobs"] for s in stats), "rnw s", stats[0]["t_rnw_s"])


@pytest.mark.parametrize("order", ["natural", "random", "exact_cost", "estimate"])
def test_orders_and_plain_agree(hperm, ctx, order):
    items = W.config_n60(3)
    mats = [A for _, A in items]
    say("order", order)
    ctx.set_opts(m_cut=24)
    try:
        J = ctx.expand(mats)
        ctx.estimate(J, 8, 11)
        tot, _, _ = ctx.run(J, order, True)
        assert tot == [int(GOLDEN[name]) for name, _ in items]
        if order == "natural":
            tot2, _, _ = ctx.run(J, order, False)
            assert tot2 == tot
    finally:
        ctx.set_opts(m_cut=20)


def test_estimate_seed_does_not_change_result(hperm, ctx):
    items = W.config_n60(1)
    mats = [A for _, A in items]
    say("estimate seeds")
    ctx.set_opts(m_cut=24)
    try:
        J = ctx.expand(mats)
        out = []
        for seed in (1, 2, 99):
            ctx.estimate(J, 4, seed)
            out.append(ctx.run(J, "estimate", True)[0])
    finally:
        ctx.set_opts(m_cut=20)
    assert out[0] == out[1] == out[2] == [int(GOLDEN[n]) for n, _ in items]


# ------------------------------------------------------------------ edge cases
def test_edge_cases(hperm, ctx):
    say("edge cases")
    Z = np.ones((6, 6), int)
    Z[:, 3] = 0
    P = np.zeros((50, 50), int)
    P[np.arange(50), np.random.default_rng(0).permutation(50)] = 1
    D = np.diag([3, 5, 7, 11, 13, 17, 19, 23])
    cases = [np.zeros((0, 0), int), np.array([[5]]), np.array([[1, 2], [3, 4]]), Z, np.eye(70, dtype=int), P, D]
    want = [1, 5, 10, 0, 1, 1, 3 * 5 * 7 * 11 * 13 * 17 * 19 * 23]
    assert ctx.permanent_batch(cases) == want
    assert hperm.permanent(np.array([[2, 1], [1, 2]])) == 5


def test_invalid_inputs_raise(hperm, ctx):
    say("invalid inputs")
    with pytest.raises(hperm.HpermError) as e:
        ctx.permanent(np.full((3, 3), 1 << 23))
    assert e.value.status == -1
    with pytest.raises(hperm.HpermError) as e:
        ctx.permanent_csr(129, np.zeros(130, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint32))
    assert e.value.status == -1


def test_caller_arena(hperm):
    """Device memory from a torch tensor: same values; an arena that is too small reports
    NOMEM with the bytes needed."""
    say("arena")
    mats = W.config_n24(range(3))
    c = hperm.Context({"m_cut": 12, "split_order": 0})
    try:
        c.set_arena(4096)
        with pytest.raises(hperm.HpermError) as e:
            c.permanent_batch(mats)
        assert e.value.status == -4
        need = c.arena_required()
        assert need > 4096
        c.set_arena(need * 4)
        assert c.permanent_batch(mats) == [int(GOLDEN[f"cubic24_seed{s}"]) for s in range(3)]
    finally:
        c.close()


# ------------------------------------------------------------------ estimator
def test_estimate_matches_oracle(hperm, ctx):
    """FP32 KKLLL keys against the float64 oracle with the same counter-based draws.

    Tolerance: the key is log(mean |det B|^2); with m <= 10 and unit-modulus entries the
    FP32 elimination gives relative errors of order m^2 * 2^-24 (about 1e-5) on the
    dominant trials, so 2e-3 absolute on the log-mean is a wide margin."""
    mats = [leaf_like(m, 300 + m, k=3) for m in (2, 4, 6, 8, 10)]
    say("estimate parity")
    J = ctx.jobs_from_dense(mats)
    keys = ctx.estimate(J, 16, 12345)
    for job, (A, key) in enumerate(zip(mats, keys)):
        want = kkl_key(A, 16, 12345, job)
        assert abs(float(key) - want) < 2e-3, (job, key, want)


def test_estimate_matches_oracle_larger_orders(hperm, ctx):
    """The same for the estimator's order buckets 17..20 and 21..24 (orders 17, 20, 22, 24).

    FP32 rounding grows like m^2 * 2^-24 (about 3e-5 at m = 24), still far inside 2e-3."""
    mats = [leaf_like(m, 350 + m, k=3) for m in (17, 20, 22, 24)]
    say("estimate parity, orders 17..24")
    J = ctx.jobs_from_dense(mats)
    keys = ctx.estimate(J, 16, 777)
    for job, (A, key) in enumerate(zip(mats, keys)):
        want = kkl_key(A, 16, 777, job)
        assert abs(float(key) - want) < 2e-3, (job, key, want)


def test_estimate_matches_oracle_buckets_32_40(hperm, ctx):
    """The estimator's order buckets 25..32 (32 lanes per trial) and 33..40 (64 lanes per
    trial, the pivot search crossing 32-lane halves): orders 25, 28, 32, 33, 36 and 40.

    FP32 rounding grows like m^2 * 2^-24 (about 1e-4 at m = 40), inside 2e-3."""
    mats = [leaf_like(m, 370 + m, k=3) for m in (25, 28, 32, 33, 36, 40)]
    say("estimate parity, orders 25..40")
    J = ctx.jobs_from_dense(mats)
    keys = ctx.estimate(J, 8, 4242)
    for job, (A, key) in enumerate(zip(mats, keys)):
        want = kkl_key(A, 8, 4242, job)
        assert abs(float(key) - want) < 2e-3, (job, A.shape[0], key, want)


def test_wide_rings_on_expanded_problems(hperm):
    """Problems whose expansion yields mod-2^128 and residue-ring jobs (a random 4-regular graph
    on 40 vertices; a 3-permutation union on 38 vertices with values 1..6): every residue-ring
    and mod-2^128 job of the union and a sample of the graph's jobs equal the oracle's
    permanent of the job's sub-matrix, and the totals equal the oracle, on the R-NW path, with
    the device continuation of H_per and on the device-expansion path."""
    Q = W.random_quartic_matrix(40, 3)
    U = W.permutation_union_matrix(38, 3, 6, 1, 6)
    want = [native.hper_batch([Q], threads=8)[0], per_dp(U)]
    for split in (0, 12):
        c = hperm.Context({"split_order": split, "device_expand": 0})
        try:
            J = c.expand([Q, U])
            d = J.describe()
            say("wide rings, split", split, "jobs", len(d["m"]), np.unique(d["arith"], return_counts=True))
            assert {2, 3} <= set(d["arith"].tolist())
            tot, pj, _ = c.run(J, "natural", True, per_job=True)
            assert tot == want
            idx_u = [k for k in range(len(pj)) if d["problem"][k] == 1]
            rng = np.random.default_rng(split)
            idx_q = [k for k in range(len(pj)) if d["problem"][k] == 0]
            wide_q = [k for k in idx_q if d["arith"][k] == 2]
            pick = idx_u + sorted(rng.choice(wide_q, 24, replace=False).tolist()) + sorted(rng.choice(idx_q, 8, replace=False).tolist())
            mats = [J.matrix(k).astype(np.int64).tolist() for k in pick]
            assert [pj[k] for k in pick] == native.ryser_batch(mats, threads=8)
        finally:
            c.close()
    c = hperm.Context()   # the default path: the graph on the device (the union's bound, above 2^102, keeps it on the host)
    try:
        assert c.permanent_batch([Q, U]) == want
        assert [l["variant"] for l in c.last_launches()].count(4) == 1
    finally:
        c.close()


def test_estimate_tracks_permanent(hperm, ctx):
    """With many trials the key approaches log per of the pattern (the estimator is unbiased)."""
    say("estimate vs per")
    pats = [(leaf_like(10, 400 + s, k=2 + s % 4) > 0).astype(np.uint32) for s in range(8)]
    J = ctx.jobs_from_dense(pats)
    keys = ctx.estimate(J, 2048, 7)
    for A, key in zip(pats, keys):
        p = per_ryser(A)
        assert abs(float(key) - math.log(p)) < 0.6


# ------------------------------------------------------------------ batched n = 80 graphs
def test_n80_batch_end_to_end(hperm):
    """The batched configuration: 8 random cubic girth>=5 graphs on 80 vertices in one batch
    (3.0M jobs of order 20 per graph, 1.3e13 subset-terms in all), exact against the stored
    oracle values; the LPT and random queue orders agree."""
    items = W.config_n80(8)
    say("n80 batch: expand 8 graphs")
    c = hperm.Context({"m_cut": 20, "max_table_mib": 32768, "split_order": 0})
    try:
        J = c.expand([A for _, A in items])
        nj, npb = J.info()
        say("n80 jobs", nj)
        c.estimate(J, 8, 1)
        tot, _, _ = c.run(J, "estimate", True)
        want = [int(GOLDEN[name]) for name, _ in items]
        assert tot == want
        say("n80 rnw ms", sum(L["ms"] for L in c.last_launches()))
        tot2, _, _ = c.run(J, "random", True)
        assert tot2 == want
    finally:
        c.close()


@pytest.mark.parametrize("chunk", [1, 2, 5])
def test_paired_walk_small_chunks(hperm, chunk):
    """Jobs of cubic graphs take the paired walk (column 0 reaching two or three rows, some
    jobs transposed) at lane chunks of 2 Gray indices, and the four-step walks (column 0 on
    two or three rows, column 1 on rows disjoint from them) at chunks of 4 and 32; with chunks
    of 2 and 4 indices the pair or block straddles the lane-dependent direction of the chunk's
    last column. Job by job against the oracle."""
    A = W.random_cubic_matrix(24, 5)
    say("paired walk, chunk", chunk)
    c = hperm.Context({"m_cut": 14, "chunk_log2": chunk, "split_order": 0})
    try:
        J = c.expand([A])
        totals, per_job, _ = c.run(J, "natural", True, per_job=True)
        variants = {L["variant"] for L in c.last_launches()}
    finally:
        c.close()
    assert per_job == native.ryser_batch(expand_leaves(A, 14), threads=8)
    assert totals == [int(GOLDEN["cubic24_seed5"])]
    if chunk >= 2:
        assert {6, 7} <= variants   # the four-step walks need lane chunks of four steps
    else:
        assert variants & {1, 2} and not variants & {6, 7}


def test_largest_orders_and_sizes(hperm, ctx):
    """Jobs of order 40 (the largest) and inputs of order 128 (the largest): closed forms
    per(a I + P) = a^n + 1 for the cyclic shift P, and the 3-band circulant I + P + P^2
    against the oracle; an input whose proven bound exceeds 2^180 is refused."""
    say("largest orders")
    n40 = [3 * np.eye(40, dtype=np.uint32) + np.roll(np.eye(40, dtype=np.uint32), 1, axis=1),
           sum(np.roll(np.eye(40, dtype=np.uint32), s, axis=1) for s in range(3))]
    J = ctx.jobs_from_dense(n40)
    assert list(J.describe()["m"]) == [40, 40]
    totals, _, _ = ctx.run(J, "natural", True)
    assert totals[0] == 3 ** 40 + 1
    assert totals[1] == native.hper_batch([n40[1]])[0]
    say("largest inputs")
    big = [np.eye(128, dtype=np.uint32) + np.roll(np.eye(128, dtype=np.uint32), 1, axis=1)]
    assert ctx.permanent_batch(big) == [2]
    with pytest.raises(hperm.HpermError) as e:
        ctx.permanent(2 * np.eye(128, dtype=np.uint32) + np.roll(np.eye(128, dtype=np.uint32), 1, axis=1))
    assert e.value.status == -2


def test_job_timing(hperm):
    """time_jobs = 1: every job of a timed persistent run gets positive work cycles, the values
    are unchanged, and jobs with 64 times the subset-terms take many times longer."""
    say("job timing")
    c = hperm.Context({"time_jobs": 1, "split_order": 0})
    try:
        mats = [leaf_like(m, 500 + i, k=3) for i, m in enumerate((14, 20, 14, 20))]
        J = c.jobs_from_dense(mats)
        totals, per_job, _ = c.run(J, "natural", True, per_job=True)
        cyc = J.cycles()
        assert per_job == native.ryser_batch(mats, threads=8)
        assert (cyc > 0).all()
        assert min(cyc[1], cyc[3]) > 10 * max(cyc[0], cyc[2]), cyc
        c.set_opts(time_jobs=0)
        totals2, _, _ = c.run(J, "natural", True)
        assert totals2 == totals
        assert (J.cycles() == cyc).all()   # an untimed run keeps the last timing
    finally:
        c.close()
