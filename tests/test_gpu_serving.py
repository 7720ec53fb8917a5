"""Serving (continuous batching with memory admission) through the C ABI, against the oracle.

Each served request must come back bit-identical to the oracle's per(A) and to the blocking
call, whatever batch it was packed into. Inputs are seeded mixed request streams from
``workloads.serving_requests`` (3-regular, 4-regular and small-integer sparse matrices).
"""
import math
import sys
import time

import numpy as np
import pytest

import workloads as W
from oracle import native

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def stream(n_requests, seed, n_lo=12, n_hi=32):
    reqs = W.serving_requests(n_requests, seed, n_lo, n_hi)
    for _, A in reqs:
        # the C oracle works modulo 2^128: keep every permanent provably below that
        assert sum(math.log2(max(int(s), 1)) for s in A.sum(axis=1)) < 127
    return [A for _, A in reqs]


def test_serving_mixed_stream_matches_oracle(hperm):
    mats = stream(30, 5)
    want = native.hper_batch(mats, threads=8)
    say("serving mixed stream", len(mats))
    c = hperm.Context({"m_cut": 16, "split_order": 0})
    try:
        c.serve_start(64, 64 << 20)
        tickets = [c.submit(A) for A in mats]
        assert all(t is not None for t in tickets)
        got = [c.wait(t, 120.0) for t in tickets]
        c.serve_stop()
        assert [v for v, _ in got] == want
        # the blocking call on the same context gives the same values
        assert c.permanent_batch(mats) == want
        for _, st in got:
            assert 0.0 <= st["t_expand_s"] <= st["t_total_s"]
    finally:
        c.close()


def test_serving_arrivals_over_time(hperm):
    """Requests arriving while earlier batches run (Poisson gaps) still come back exact."""
    mats = stream(24, 9, 16, 30)
    want = native.hper_batch(mats, threads=8)
    gaps = np.diff(np.concatenate([[0.0], W.poisson_arrivals(len(mats), 400.0, 3)]))
    say("serving arrivals", len(mats))
    c = hperm.Context({"m_cut": 14, "split_order": 0})
    try:
        c.serve_start(64, 32 << 20)
        tickets = []
        for A, g in zip(mats, gaps):
            time.sleep(float(g))
            tickets.append(c.submit(A))
        got = [c.wait(t, 120.0)[0] for t in tickets]
        assert got == want
    finally:
        c.close()


def test_serving_small_arena_admission(hperm):
    """A 1 MiB arena admits only a few requests per batch: many batches, same values. A request
    whose own buffers exceed the arena completes with NOMEM and does not block the others."""
    mats = stream(12, 21, 16, 28)
    want = native.hper_batch(mats, threads=8)
    big = W.config_n60(1)[0][1]
    say("serving small arena")
    c = hperm.Context({"m_cut": 16, "split_order": 0})
    try:
        c.serve_start(32, 1 << 20)
        tb = c.submit(big)
        tickets = [c.submit(A) for A in mats]
        got = [c.wait(t, 120.0)[0] for t in tickets]
        assert got == want
        with pytest.raises(hperm.HpermError) as e:
            c.wait(tb, 120.0)
        assert e.value.status == -4
    finally:
        c.close()


def test_serving_slots_cancel_and_errors(hperm):
    A = stream(1, 2, 20, 20)[0]
    want = native.hper_batch([A])[0]
    say("serving slots/cancel")
    c = hperm.Context({"m_cut": 16, "split_order": 0})
    try:
        with pytest.raises(hperm.HpermError):
            c.poll(1)   # not serving
        c.serve_start(2, 8 << 20)
        with pytest.raises(hperm.HpermError):
            c.serve_start(2, 8 << 20)   # already serving
        with pytest.raises(hperm.HpermError):
            c.permanent(A)   # blocking calls are refused while serving
        with pytest.raises(hperm.HpermError):
            c.set_opts(m_cut=12)
        t1 = c.submit(A)
        t2 = c.submit(A)
        assert c.submit(A) is None   # both request slots are live until their results are taken
        c.cancel(t1)
        with pytest.raises(hperm.HpermError) as e:
            c.wait(t1, 120.0)
        assert e.value.status == -6
        assert c.wait(t2, 120.0)[0] == want
        with pytest.raises(hperm.HpermError):
            c.poll(t2)   # a result is taken once
        t3 = c.submit(A)
        r = None
        deadline = time.time() + 120
        while r is None and time.time() < deadline:
            r = c.poll(t3)
            time.sleep(0.002)
        assert r is not None and r[0] == want
        with pytest.raises(hperm.HpermError):
            c.submit(np.full((3, 3), 1 << 23))   # entry beyond the limit
        c.serve_stop()
        c.serve_start(4, 8 << 20)   # a context can serve again
        assert c.wait(c.submit(A), 120.0)[0] == want
    finally:
        c.close()


def test_serving_edge_cases(hperm):
    Z = np.ones((6, 6), int)
    Z[:, 3] = 0
    cases = [np.zeros((0, 0), int), np.array([[5]]), Z, np.array([[1, 2], [3, 4]]), np.ones((22, 22), int)]
    want = [1, 5, 0, 10, math.factorial(22)]
    say("serving edge cases")
    c = hperm.Context()
    try:
        c.serve_start(8, 8 << 20)
        got = [c.wait(c.submit(A), 120.0)[0] for A in cases]
        assert got == want
    finally:
        c.close()


def test_serving_device_lane_and_work_limit(hperm):
    """Requests above the device expansion's order run in the device lane (grouped by order,
    overlapping the host batches) and come back equal to the oracle; with a work limit, a
    request whose estimated work is far beyond it is refused with HPERM_E_TOOBIG while the
    others are served."""
    mats = [W.random_cubic_matrix(n, 40 + n) for n in (24, 30, 30, 36, 44)]
    mats += [W.random_quartic_matrix(n, 50 + n) for n in (20, 26, 30)]
    mats += [W.permutation_union_matrix(n, 3, 60 + n, 1, 3) for n in (18, 28, 34)]
    want = native.hper_batch(mats, threads=8)
    say("serving device lane", len(mats))
    c = hperm.Context({"split_order": 12, "device_expand": 22, "serve_limit_ms": 2000})
    try:
        c.serve_start(64, 256 << 20)
        tickets = [c.submit(A) for A in mats]
        big = c.submit(W.random_cubic_matrix(100, 0))   # about 30 s of GPU time
        got = [c.wait(t, 120.0) for t in tickets]
        with pytest.raises(hperm.HpermError) as e:
            c.wait(big, 60.0)
        assert e.value.status == -9
        c.serve_stop()
    finally:
        c.close()
    assert [v for v, _ in got] == want
    lanes = [st["max_m"] for _, st in got]
    assert 22 in lanes and any(m != 22 for m in lanes)


def test_serving_large_requests_equal_oracle(hperm):
    """The benchmark's graphs as serving requests at full size: the 17 cubic graphs on 60
    vertices and the 8 on 80 vertices (the device lane), interleaved with small requests (the
    batch path), all in flight together; every result equals the oracle's stored value (and the
    small ones the C oracle)."""
    import json
    import os
    golden = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                         "oracle_values.json")))
    big = W.config_n60(16) + W.config_n80(8)
    small = stream(12, 23)
    want_small = native.hper_batch(small, threads=8)
    say("serving large requests", len(big), "small", len(small))
    c = hperm.Context({"split_order": 12, "device_expand": 22, "device_expand_mib": 4096})
    try:
        c.serve_start(64, 256 << 20)
        tickets = []
        for k, (_, A) in enumerate(big):
            tickets.append(c.submit(A))
            if k < len(small):
                tickets.append(c.submit(small[k]))
        got = [c.wait(t, 300.0)[0] for t in tickets]
        c.serve_stop()
    finally:
        c.close()
    want = []
    for k, (name, _) in enumerate(big):
        want.append(int(golden[name]))
        if k < len(small):
            want.append(want_small[k])
    assert got == want
