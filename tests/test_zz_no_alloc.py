"""The no-allocation entry point (hperm_permanent_dense_noalloc) through the C ABI: its
value equals hperm_permanent_dense's on the same matrix, for every ring, on two calls in a
row with the second input smaller (the fixed scratch array keeps the first call's
contents and must be cleared), plus its edge cases and its size limit."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair_cases():
    rng = np.random.default_rng(5)
    a22 = (rng.integers(0, 4, size=(22, 22)) * (rng.random((22, 22)) < 0.3)).astype(np.uint32)
    np.fill_diagonal(a22, 1)
    a9 = rng.integers(0, 6, size=(9, 9)).astype(np.uint32)
    a12 = W.permutation_union_matrix(12, 4, 3, 1, 5)
    a16 = W.permutation_union_matrix(16, 5, 7, 1, 9)
    return [
        ("w64", a22, a9),
        ("w128", np.ones((24, 24), np.uint32), a12),
        ("res", 2 * np.ones((30, 30), np.uint32), a16),
    ]


@pytest.mark.parametrize("ring,big,small", _pair_cases(), ids=lambda x: x if isinstance(x, str) else None)
def test_noalloc_equals_dense_entry_on_two_calls(hperm, ring, big, small):
    ctx = hperm.Context({"m_cut": 20})
    try:
        got = [ctx.permanent_dense_noalloc(big), ctx.permanent_dense_noalloc(small)]
        want = [ctx.permanent_dense(big), ctx.permanent_dense(small)]
        assert got == want, (ring, got, want)
        # and the same pair again, in the other order
        assert ctx.permanent_dense_noalloc(small) == want[1]
        assert ctx.permanent_dense_noalloc(big) == want[0]
    finally:
        ctx.close()
    if ring == "w128":
        assert got[0] == math.factorial(24)
    if ring == "res":
        assert got[0] == 2 ** 30 * math.factorial(30)


def test_noalloc_edge_cases_and_limit(hperm):
    ctx = hperm.Context()
    try:
        assert ctx.permanent_dense_noalloc(np.zeros((0, 0), np.uint32)) == 1
        z = np.ones((6, 6), np.uint32)
        z[:, 3] = 0
        assert ctx.permanent_dense_noalloc(z) == 0
        assert ctx.permanent_dense_noalloc(np.array([[7]], np.uint32)) == 7
        assert ctx.permanent_dense_noalloc(np.array([[1, 2], [3, 4]], np.uint32)) == 10
        with pytest.raises(hperm.HpermError) as e:
            ctx.permanent_dense_noalloc(np.ones((41, 41), np.uint32))
        assert e.value.status == -1
        # a context of its own shares the array: still exact after the error
        c2 = hperm.Context()
        try:
            assert c2.permanent_dense_noalloc(np.ones((10, 10), np.uint32)) == math.factorial(10)
        finally:
            c2.close()
        assert ctx.permanent_dense_noalloc(np.ones((8, 8), np.uint32)) == math.factorial(8)
    finally:
        ctx.close()
