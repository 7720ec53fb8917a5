"""The grouped Gray-code sums that the R-NW kernels take in place of single steps, checked on
the host with exact integers against the oracle's permanent (no GPU needed).

The doubled Nijenhuis-Wilf form of Ryser's formula (the Introduction's R-NW): with one fixed
column and Gray columns c_0 .. c_{m-2}, the row values at Gray code g are
f_i(g) = 2 a_{i,fixed} - r_i + 2 sum over the set bits j of g of a_{i,c_j} (r_i the row sum),
V = sum_k (-1)^k prod_i f_i(g(k)) over the reflected code g(k) = k xor (k >> 1), and
per(A) = (-1)^(m-1) V / 2^(m-1). The kernels sum two consecutive terms at once when Gray
column 0 reaches only the rows P (the paired walks), and four when Gray column 0 reaches only
the rows A and Gray column 1 only rows B disjoint from A (the four-step walks):
  terms 2p, 2p+1:        +-(prod_P (g + d) - prod_P g) * (other rows), plus when column 0 is
                         set in term 2p;
  terms 4q .. 4q+3:      (-1)^q (A0 - A1)(B0 - B1) * (other rows),
where g holds the rows without columns 0 and 1, d the column's doubled entries, A0/A1 (B0/B1)
the products over A (B) without/with column 0 (column 1)."""
import numpy as np
import pytest

import workloads as W
from oracle import per_brute, per_ryser


def gray_rows(A, gray, fixed):
    """f_i(g(k)) for every k (rows of the result) and the Gray codes themselves."""
    A = np.asarray(A, dtype=np.int64)
    m = A.shape[0]
    k = np.arange(1 << (m - 1), dtype=np.int64)
    g = k ^ (k >> 1)
    base = 2 * A[:, fixed] - A.sum(1)
    bits = ((g[:, None] >> np.arange(m - 1)[None, :]) & 1)            # (K, m-1)
    f = base[None, :] + 2 * bits @ A[:, gray].T                         # (K, m)
    return f, g


def per_from_v(v, m):
    assert v % (1 << (m - 1)) == 0
    return (-1) ** (m - 1) * (v >> (m - 1))


def nw_single_steps(A, gray, fixed):
    f, _ = gray_rows(A, gray, fixed)
    sign = 1 - 2 * (np.arange(f.shape[0]) & 1)
    return per_from_v(int((sign * f.prod(1)).sum()), f.shape[1])


def nw_pairs(A, gray, fixed, P):
    """Pairs around Gray column 0, whose nonzeros lie in rows P only."""
    A = np.asarray(A, dtype=np.int64)
    f, g = gray_rows(A, gray, fixed)
    m = A.shape[0]
    d = 2 * A[:, gray[0]]
    other = [i for i in range(m) if i not in P]
    v = 0
    for p in range(f.shape[0] // 2):
        t = 2 * p
        row = f[t] - d * (g[t] & 1)                 # rows without column 0
        x = int(np.prod(row[P] + d[P])) - int(np.prod(row[P]))
        v += (1 if g[t] & 1 else -1) * x * int(np.prod(row[other]))
    return per_from_v(v, m)


def nw_blocks(A, gray, fixed, RA, RB, sign_q=True):
    """Blocks of four steps over Gray columns 0 (rows RA only) and 1 (rows RB only)."""
    A = np.asarray(A, dtype=np.int64)
    f, g = gray_rows(A, gray, fixed)
    m = A.shape[0]
    d0, d1 = 2 * A[:, gray[0]], 2 * A[:, gray[1]]
    other = [i for i in range(m) if i not in RA and i not in RB]
    v = 0
    for q in range(f.shape[0] // 4):
        t = 4 * q
        row = f[t] - d0 * (g[t] & 1) - d1 * ((g[t] >> 1) & 1)   # columns 0 and 1 out
        a0, a1 = int(np.prod(row[RA])), int(np.prod(row[RA] + d0[RA]))
        b0, b1 = int(np.prod(row[RB])), int(np.prod(row[RB] + d1[RB]))
        s = (-1) ** q if sign_q else 1
        v += s * (a0 - a1) * (b0 - b1) * int(np.prod(row[other]))
    return per_from_v(v, m)


def structured(m, a, nb, seed):
    """An m x m integer matrix (entries 0..4) whose column c0 has nonzeros only in the rows RA
    (|RA| = a) and column c1 only in rows RB (|RB| = nb) disjoint from RA; rows and columns in
    random positions."""
    rng = np.random.default_rng(seed)
    A = rng.integers(0, 5, (m, m))
    rows = rng.permutation(m)
    RA, RB = sorted(rows[:a].tolist()), sorted(rows[a:a + nb].tolist())
    c0, c1, fixed = rng.choice(m, 3, replace=False).tolist()
    A[:, c0] = 0
    A[RA, c0] = rng.integers(1, 5, a)
    A[:, c1] = 0
    A[RB, c1] = rng.integers(1, 5, nb)
    rest = [j for j in rng.permutation(m).tolist() if j not in (c0, c1, fixed)]
    return A, [c0, c1] + rest, fixed, RA, RB


@pytest.mark.parametrize("seed", range(8))
def test_single_steps_pairs_and_blocks_give_the_permanent(seed):
    m = 5 + seed % 4
    a, nb = 2 + seed % 2, 1 + seed % 3
    A, gray, fixed, RA, RB = structured(m, a, nb, 100 + seed)
    want = per_brute(A.tolist()) if m <= 8 else per_ryser(A.tolist())
    assert nw_single_steps(A, gray, fixed) == want
    assert nw_pairs(A, gray, fixed, RA) == want
    assert nw_blocks(A, gray, fixed, RA, RB) == want


def test_block_sign_matters():
    """Dropping the (-1)^q of the blocks changes the result: the identity is not vacuous."""
    wrong = 0
    for seed in range(8):
        A, gray, fixed, RA, RB = structured(7, 2, 3, 200 + seed)
        if nw_blocks(A, gray, fixed, RA, RB, sign_q=False) != per_ryser(A.tolist()):
            wrong += 1
    assert wrong >= 6


def test_blocks_on_the_expansions_jobs():
    """Jobs of the host expansion whose first two Gray columns have the four-step shape: the
    block sums over the job's own Gray order (rows as stored: column 0 on rows 0..a-1,
    column 1 on rows of a..a+2) give the oracle's permanent of the job."""
    import paper_1112_6072_amd as hp
    c = hp.Context({"m_cut": 12}, host_only=True)
    J = c.expand([W.random_cubic_matrix(22, 3)])
    seen = {2: 0, 3: 0}
    for k in range(J.info()[0]):
        B = J.matrix(k).astype(np.int64)
        m = B.shape[0]
        r0 = np.nonzero(B[:, 0])[0].tolist()
        r1 = np.nonzero(B[:, 1])[0].tolist()
        a = len(r0)
        if a not in (2, 3) or r0 != list(range(a)) or not r1 or min(r1) < a or max(r1) >= a + 3:
            continue
        gray, fixed = list(range(m - 1)), m - 1
        RB = list(range(a, a + 3))
        assert nw_blocks(B, gray, fixed, r0, RB) == per_ryser(B.tolist())
        seen[a] += 1
        if min(seen.values()) >= 2:
            break
    assert min(seen.values()) >= 1


def fp32_block_diffs(row, d0, d1, RA, RB):
    """A1 - A0 and B1 - B0 as the kernels take them for rows of at most three values: the
    product of the first two in FP32, then the third product and the difference fused (one
    rounding of the exact value), each converted to an integer."""
    def diff(idx, d):
        h = [np.float32(row[i] + d[i]) for i in idx]
        g = [np.float32(row[i]) for i in idx]
        p0 = np.float32(g[0] * g[1]) if len(idx) > 1 else g[0]
        p1 = np.float32(h[0] * h[1]) if len(idx) > 1 else h[0]
        if len(idx) == 3:
            # fused multiply-add: the exact p1 * h2 - p0 * g2 rounded once to FP32
            q0 = np.float32(float(p0) * float(g[2]))
            return int(np.float32(float(p1) * float(h[2]) - float(q0)))
        return int(np.float32(float(p1) - float(p0)))
    return diff(RA, d0), diff(RB, d1)


@pytest.mark.parametrize("a", [2, 3])
def test_fp32_block_sums_exact_below_2_7(a):
    """With rows of A and B whose values stay below 2^7 in magnitude (row sums up to 127), the
    FP32 block differences equal the integer ones in every block and fit the 24-bit
    multiplier's operands (below 2^23); larger row sums break one or the other."""
    rng = np.random.default_rng(40 + a)
    m = 9
    for trial in range(6):
        A = np.zeros((m, m), np.int64)
        for i in range(m):
            cols = rng.choice(m, 3, replace=False)
            A[i, cols] = rng.integers(1, 32, 3)
        A[:, 0] = 0
        A[:a, 0] = rng.integers(1, 32, a)
        A[:, 1] = 0
        A[a:a + 3, 1] = rng.integers(1, 32, 3)   # at most 4 entries below 32: row sums below 2^7
        assert A.sum(1).max() < 128
        RA, RB = list(range(a)), list(range(a, a + 3))
        f, g = gray_rows(A, list(range(m - 1)), m - 1)
        d0, d1 = 2 * A[:, 0], 2 * A[:, 1]
        for q in range(f.shape[0] // 4):
            t = 4 * q
            row = f[t] - d0 * (g[t] & 1) - d1 * ((g[t] >> 1) & 1)
            assert np.abs(row[:a + 3]).max() < 128 and np.abs((row + d0)[:a]).max() < 128
            da, db = fp32_block_diffs(row, d0, d1, RA, RB)
            assert da == int(np.prod(row[RA] + d0[RA])) - int(np.prod(row[RA]))
            assert db == int(np.prod(row[RB] + d1[RB])) - int(np.prod(row[RB]))
            assert abs(da) < 1 << 22 and abs(db) < 1 << 22
    # past the bound: at row sums of 2^8 a difference of two products of three (-255^3 against
    # 255^3) leaves the 24-bit multiplier's operand range, and at 2^9 an odd product of three
    # no longer fits FP32's 24-bit significand
    assert 2 * 255 ** 3 >= 1 << 23
    big = [np.float32(511), np.float32(509), np.float32(503)]
    assert int(np.float32(float(np.float32(big[0] * big[1])) * float(big[2]))) != 511 * 509 * 503
