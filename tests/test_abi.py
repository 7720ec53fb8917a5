"""The C-ABI library on the CPU: it loads, exports every declared call, and its host stages
(validation, expansion, arithmetic-mode choice) behave as documented. No GPU work here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import expand_leaves

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hperm.h")


@pytest.fixture(scope="module")
def hp():
    import paper_1112_6072_amd as hp
    return hp


def declared_calls():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hperm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call(hp):
    lib = ctypes.CDLL(hp.LIB_PATH)
    calls = declared_calls()
    assert len(calls) >= 25
    for name in calls:
        assert hasattr(lib, name), name
    assert set(calls) == set(hp.EXPORTED)


def test_version_and_defaults(hp):
    assert hp.version() == (1, 0)
    d = hp.default_opts()
    assert d["m_cut"] == 20 and d["s_leaf"] == 5 and d["persistent"] == 1 and d["trials"] == 32


def test_status_strings(hp):
    for s in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8):
        assert hp._lib.hperm_status_string(s).decode() not in ("", "unknown status")


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("m_cut", [8, 12, 16])
def test_expansion_matches_oracle_job_sequence(hp, seed, m_cut):
    """The host expansion and the oracle's expansion follow the same rule: same jobs, same order."""
    A = W.random_cubic_matrix(24, seed) if seed < 3 else W.permutation_union_matrix(20, 3, seed, 1, 5)
    ctx = hp.Context({"m_cut": m_cut}, host_only=True)
    d = ctx.expand([A]).describe()
    leaves = expand_leaves(A, m_cut)
    assert list(d["m"]) == [len(x) for x in leaves]


def test_expansion_s_leaf_and_cap(hp):
    """Dense nodes (every line >= s_leaf nonzeros) stop early when their order is <= m_cap."""
    A = W.random_sparse_int_matrix(18, 6, 3, 1, 3)
    for s_leaf, m_cap in ((5, 18), (5, 16), (7, 16)):
        ctx = hp.Context({"m_cut": 8, "s_leaf": s_leaf, "m_cap": m_cap}, host_only=True)
        d = ctx.expand([A]).describe()
        leaves = expand_leaves(A, 8, s_leaf, m_cap)
        assert list(d["m"]) == [len(x) for x in leaves]
        assert d["m"].max() <= m_cap


def test_expansion_is_thread_count_independent(hp):
    mats = [A for _, A in W.config_n60(2)]
    ref = None
    for th in (1, 3, 8):
        d = hp.Context({"m_cut": 26, "host_threads": th}, host_only=True).expand(mats).describe()
        cur = (list(d["m"]), list(d["problem"]), list(d["arith"]))
        assert ref is None or cur == ref
        ref = cur


def test_arith_mode_choice_from_bounds(hp):
    ctx = hp.Context(host_only=True)
    # J_12: per = 12! ~ 2^28.8, plus 12 bits of NW doubling -> 64-bit ring
    # J_20: 20! ~ 2^61.1 + 20 -> 128-bit ring; J_34: 34! ~ 2^127.8 -> residues
    d = ctx.jobs_from_dense([np.ones((12, 12)), np.ones((20, 20)), np.ones((34, 34))]).describe()
    assert list(d["arith"]) == [hp.ARITH_W64, hp.ARITH_W128, hp.ARITH_RES]
    # forcing a ring narrower than the bound is refused
    with pytest.raises(hp.HpermError) as e:
        hp.Context({"arith": "w64"}, host_only=True).jobs_from_dense([np.ones((20, 20))])
    assert e.value.status == -2
    d = hp.Context({"arith": "res"}, host_only=True).jobs_from_dense([np.ones((5, 5))]).describe()
    assert list(d["arith"]) == [hp.ARITH_RES]


def test_gray_order_for_the_four_step_walks(hp):
    """For a mod 2^64 job whose first Gray column reaches at most three rows, Gray column 1 is
    the sparsest column (of at most three rows) that avoids those rows when one exists, and
    the job's rows are ordered column 0's first, then column 1's (the layout the kernels'
    four-step walks take: A = rows 0..a-1, B = rows of a..a+2)."""
    shapes = {2: 0, 3: 0}
    for seed in range(6):
        ctx = hp.Context({"m_cut": 14}, host_only=True)
        J = ctx.expand([W.random_cubic_matrix(26, seed)])
        d = J.describe()
        for k in range(len(d["m"])):
            A = J.matrix(k)
            m = A.shape[0]
            r0 = set(np.nonzero(A[:, 0])[0])
            a = len(r0)
            if d["arith"][k] != hp.ARITH_W64 or a > 3 or m < 5:
                continue
            assert r0 == set(range(a))
            cand = [len(np.nonzero(A[:, j])[0]) for j in range(1, m - 1)
                    if not r0 & set(np.nonzero(A[:, j])[0]) and 1 <= len(np.nonzero(A[:, j])[0]) <= 3]
            if not cand:
                continue
            r1 = set(np.nonzero(A[:, 1])[0])
            assert not r0 & r1 and len(r1) == min(cand)
            assert r1 == set(range(a, a + len(r1)))
            if a >= 2 and m >= a + 3:
                shapes[a] += 1
    assert shapes[2] > 0 and shapes[3] > 0


def test_terms_and_orders(hp):
    ctx = hp.Context({"m_cut": 14}, host_only=True)
    d = ctx.expand([W.random_cubic_matrix(24, 0)]).describe()
    assert all(int(t) == 1 << (int(m) - 1) for m, t in zip(d["m"], d["terms"]))


@pytest.mark.parametrize("bad", ["unsorted", "dup", "range", "rowptr", "big_entry", "n"])
def test_validation_errors(hp, bad):
    ctx = hp.Context(host_only=True)
    n = 4
    rp = np.array([0, 2, 4, 6, 8], np.int32)
    ci = np.array([0, 1, 1, 2, 2, 3, 0, 3], np.int32)
    va = np.ones(8, np.uint32)
    if bad == "unsorted":
        ci[0], ci[1] = 1, 0
    elif bad == "dup":
        ci[1] = 0
    elif bad == "range":
        ci[7] = 9
    elif bad == "rowptr":
        rp[2] = 1
    elif bad == "big_entry":
        va[3] = 1 << 23
    elif bad == "n":
        n = 129
        rp = np.zeros(130, np.int32)
    h = ctypes.c_void_p()
    nn = np.array([n], np.int32)
    z = np.zeros(1, np.int64)
    st = hp._lib.hperm_expand_batch_csr(ctx.handle, 1, hp._ptr(nn), hp._ptr(z), hp._ptr(z), hp._ptr(rp),
                                        hp._ptr(ci), hp._ptr(va), ctypes.byref(h))
    assert st == -1
    assert hp._lib.hperm_last_error(ctx.handle).decode() != ""


def test_host_only_context_refuses_gpu_calls(hp):
    ctx = hp.Context(host_only=True)
    J = ctx.jobs_from_dense([np.ones((3, 3))])
    with pytest.raises(hp.HpermError) as e:
        ctx.run(J)
    assert e.value.status == -3
    with pytest.raises(hp.HpermError) as e:
        ctx.serve_start(4, 1 << 20)
    assert e.value.status == -3
    # serving calls on a context that is not serving are refused, not crashed
    assert hp._lib.hperm_poll(ctx.handle, 1, None) == -1
    assert hp._lib.hperm_cancel(ctx.handle, 1) == -1
    assert hp._lib.hperm_serve_stop(ctx.handle) == -1


def test_zero_and_empty_problems_need_no_jobs(hp):
    ctx = hp.Context(host_only=True)
    Z = np.ones((5, 5), int)
    Z[2] = 0
    J = ctx.expand([np.zeros((0, 0)), Z])
    assert J.info() == (0, 2)


def test_residue_primes_are_prime():
    import sympy
    for c in (1, 31, 45):
        assert sympy.isprime(2 ** 61 - c)
    assert math.prod(2 ** 61 - c for c in (1, 31, 45)) > 2 ** 182


def test_job_cycles_need_a_timed_run(hp):
    c = hp.Context(host_only=True)
    try:
        J = c.jobs_from_dense([np.ones((3, 3), np.uint32)])
        with pytest.raises(hp.HpermError):
            J.cycles()
        with pytest.raises(hp.HpermError):
            c.set_opts(time_jobs=2)
    finally:
        c.close()


def test_tree_estimate_exact_and_unbiased(hp):
    """Knuth's estimate of the expansion tree (host): exact for a tree without branching (a
    permutation matrix: one node per order), and close to the oracle's exact job count for
    cubic graphs (every node above the cut-off split, as expand_leaves does with no s_leaf
    stop)."""
    n = 20
    P = np.zeros((n, n), np.uint32)
    P[np.arange(n), (np.arange(n) * 7) % n] = 3
    nodes, leaves = hp.tree_estimate(P, samples=50, seed=2, split_order=8, device_expand=12)
    assert nodes[8:].tolist() == [1.0] * (n - 7) and leaves[8] == 1.0 and leaves.sum() == 1.0
    for seed in (0, 1):
        A = W.random_cubic_matrix(30, seed)
        exact = len(expand_leaves(np.asarray(A, dtype=np.int64), 12, 10 ** 9, 40))
        _, lv = hp.tree_estimate(A, samples=20000, seed=5, split_order=12, device_expand=12, m_cut=12)
        assert abs(lv.sum() - exact) <= 0.05 * exact, (lv.sum(), exact)


def test_tree_estimate_any_values(hp):
    """The tree's shape depends on the nonzero pattern only: the estimate for an integer matrix
    whose expansion leaves the exact entry range (a union of three permutations, values 1..4,
    48 vertices) equals its 0-1 pattern's with the same descents, and is close to the oracle's
    exact leaf count of the valued matrix."""
    A = W.permutation_union_matrix(48, 3, 48)
    P = (A > 0).astype(np.uint32)
    kw = dict(split_order=12, device_expand=12, m_cut=12)
    a = hp.tree_estimate(A, samples=500, seed=3, **kw)
    b = hp.tree_estimate(P, samples=500, seed=3, **kw)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    exact = len(expand_leaves(A.astype(np.int64), 12, 10 ** 9, 60))
    _, lv = hp.tree_estimate(A, samples=20000, seed=5, **kw)
    assert abs(lv.sum() - exact) <= 0.05 * exact, (lv.sum(), exact)
