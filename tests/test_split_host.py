"""Host side of the device continuation of H_per: option checks and the job sub-matrix
accessor the split parity tests hand to the oracle (no GPU needed)."""
import numpy as np
import pytest

import workloads as W
from oracle import expand_leaves, native


@pytest.fixture(scope="module")
def hp():
    import paper_1112_6072_amd as hp
    return hp


def test_split_order_checked(hp):
    c = hp.Context(host_only=True)
    for bad in (-1, 1, 6, 24, 40):
        with pytest.raises(hp.HpermError):
            c.set_opts(split_order=bad)
    c.set_opts(split_order=12, s_leaf=6)   # accepted; the device continuation is then off
    c.set_opts(s_leaf=5)
    for good in (0, 7, 12, 19, 23):
        c.set_opts(split_order=good)
    assert hp.Context(host_only=True)._opts.split_order == 12   # the default


@pytest.mark.parametrize("m_cut", [10, 14])
def test_job_matrix_is_the_expansion_leaf(hp, m_cut):
    """The stored sub-matrix of every job is a row/column permutation (or transpose) of the
    oracle's leaf: same order, same nonzero count and entry multiset, same permanent."""
    A = W.random_cubic_matrix(24, 5)
    c = hp.Context({"m_cut": m_cut}, host_only=True)
    J = c.expand([A])
    mats = [J.matrix(k).astype(np.int64) for k in range(J.info()[0])]
    leaves = [np.array(x, np.int64) for x in expand_leaves(A, m_cut)]
    assert len(mats) == len(leaves)
    key = lambda B: (B.shape[0], tuple(sorted(B.ravel().tolist())))
    assert sorted(map(key, mats)) == sorted(map(key, leaves))
    assert sorted(native.ryser_batch([B.tolist() for B in mats], threads=8)) == \
        sorted(native.ryser_batch([B.tolist() for B in leaves], threads=8))


def test_job_matrix_of_dense_jobs(hp):
    mats = [W.permutation_union_matrix(m, 3, 40 + m, 1, 5) for m in (3, 9, 17)]
    c = hp.Context(host_only=True)
    J = c.jobs_from_dense(mats)
    got = [J.matrix(k).astype(np.int64).tolist() for k in range(3)]
    assert native.ryser_batch(got, threads=4) == native.ryser_batch([A.astype(np.int64).tolist() for A in mats], threads=4)
    with pytest.raises(hp.HpermError):
        J.matrix(3)
