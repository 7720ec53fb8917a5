"""The autotuner of the persistent R-NW launches through the C ABI: tuned runs give the same
exact values as default runs (the lane chunk only regroups the same Gray indices), the tuning
table survives a JSON cache round trip, and clearing it restores the defaults."""
import json
import math
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import native

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "oracle_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_tuned_n60_equals_default_and_cache_round_trip(hperm, tmp_path):
    items = W.config_n60(4)
    mats = [A for _, A in items]
    want = [int(GOLDEN[n]) for n, _ in items]
    c = hperm.Context({"split_order": 0, "device_expand": 0})
    cache = str(tmp_path / "tune.json")
    try:
        J = c.expand(mats)
        c.estimate(J, 32, 1)
        base, pj0, _ = c.run(J, "estimate", True, per_job=True)
        say("tuning n60 groups")
        table = c.autotune(J, cache_path=cache)
        say("table", table)
        assert table and all(-3 <= e["chunk_delta"] <= 1 and e["grid_pct"] in (50, 75, 100) for e in table)
        assert all(e["ms_tuned"] <= e["ms_default"] for e in table if not e["from_cache"])
        for order in ("estimate", "natural"):
            tot, pj, _ = c.run(J, order, True, per_job=True)
            assert tot == want and pj == pj0
        assert c.permanent_batch(mats) == want
        c.tune_clear()
        assert c.run(J, "natural", True)[0] == want
    finally:
        c.close()
    saved = json.load(open(cache))
    assert len(saved) == 1 and all(len(v) == 2 for v in next(iter(saved.values())).values())
    c2 = hperm.Context({"split_order": 0, "device_expand": 0})
    try:
        loaded = c2.autotune(None, cache_path=cache)
        key = lambda e: (e["ring"], e["bucket"], e["variant"], e["chunk_delta"], e["grid_pct"])  # noqa: E731
        assert sorted(map(key, loaded)) == sorted(map(key, table))
        assert all(e["from_cache"] for e in loaded)
        assert c2.permanent_batch(mats) == want
    finally:
        c2.close()


def test_tuned_uneven_rings_equal_oracle(hperm):
    """Job-like integer matrices of orders 14..20 in the three rings: per-job values after
    tuning equal the oracle's (plain Ryser)."""
    rng = np.random.default_rng(4)
    mats = [W.permutation_union_matrix(int(m), int(rng.integers(3, 6)), 100 + i, 1, int(rng.integers(1, 9)))
            for i, m in enumerate(rng.integers(14, 21, size=40))]
    want = native.ryser_batch(mats, threads=8)
    mats += [np.ones((24, 24), np.uint32), 2 * np.ones((22, 22), np.uint32)]
    want += [math.factorial(24), 2 ** 22 * math.factorial(22)]
    c = hperm.Context({"split_order": 0, "device_expand": 0})
    try:
        J = c.jobs_from_dense(mats)
        rings = sorted(set(J.describe()["arith"].tolist()))
        say("tuning uneven jobs, rings", rings)
        table = c.autotune(J)
        assert table
        _, pj, _ = c.run(J, "natural", True, per_job=True)
        assert pj == want
        assert len(rings) >= 2
    finally:
        c.close()
