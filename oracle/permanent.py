"""Exact permanents in Python integers (oracle; test infrastructure only).

Every routine takes a square matrix (a numpy array or a list of lists of non-negative
or signed integers) and returns a Python ``int``. Nothing here is blocked, fused or
reordered beyond what the cited definition or algorithm states.

Parity pins (tests/test_oracle.py) tie each routine to facts fixed outside this file:
closed forms (per(J_k)=k!, permutation and diagonal matrices), block-diagonal
products, transpose/permutation/scaling laws, agreement between independent routes,
the 3-regular Schrijver/Bregman window, and the paper's printed per(A(C100)).
"""
from __future__ import annotations

import itertools
from collections import defaultdict


def _as_lists(A) -> list[list[int]]:
    rows = [[int(x) for x in row] for row in (A.tolist() if hasattr(A, "tolist") else A)]
    n = len(rows)
    if any(len(r) != n for r in rows):
        raise ValueError("matrix must be square")
    return rows


# --------------------------------------------------------------------------- eq. (1)
def per_brute(A) -> int:
    """The permanent by its definition (eq. 1, Introduction): the sum over all permutations
    sigma of prod_i a[i][sigma(i)]. Cost n! * n; use for n <= 9."""
    a = _as_lists(A)
    n = len(a)
    total = 0
    for sigma in itertools.permutations(range(n)):
        p = 1
        for i in range(n):
            p *= a[i][sigma[i]]
            if p == 0:
                break
        total += p
    return total


# --------------------------------------------------------------------------- R-NW
def per_ryser(A) -> int:
    """Ryser's formula (the method cited in the Introduction as the first half of R-NW):

        per(A) = (-1)^n * sum over column subsets S of (-1)^{|S|} * prod_i sum_{j in S} a[i][j].

    Subsets are enumerated in plain binary order, each row sum recomputed from scratch."""
    a = _as_lists(A)
    n = len(a)
    if n == 0:
        return 1
    total = 0
    for mask in range(1 << n):
        cols = [j for j in range(n) if mask >> j & 1]
        p = 1
        for i in range(n):
            p *= sum(a[i][j] for j in cols)
            if p == 0:
                break
        total += -p if (len(cols) & 1) else p
    return -total if (n & 1) else total


def nw_doubled_sum(A) -> int:
    """The Nijenhuis-Wilf form of Ryser's formula (the second half of R-NW, Introduction) with
    every factor doubled so that it is an integer.

    Column n (the last) is fixed. For S a subset of the first n-1 columns,
        f_i(S) = sum_{j in S or j = n} a[i][j]  -  sum_{j not in S, j != n} a[i][j],
    and the returned value is V = sum_S (-1)^{|S|} prod_i f_i(S). Nijenhuis and Wilf's
    identity per(A) = (-1)^{n-1} 2 sum_S (-1)^{|S|} prod_i (x_i + sum_{j in S} a_ij) with
    x_i = a_in - (row sum)/2, doubled in each of the n factors, gives
        V = (-1)^{n-1} * 2^{n-1} * per(A).
    Subsets are enumerated in binary order."""
    a = _as_lists(A)
    n = len(a)
    if n == 0:
        return 1
    total = 0
    for mask in range(1 << (n - 1)):
        p = 1
        for i in range(n):
            f = a[i][n - 1]
            for j in range(n - 1):
                f += a[i][j] if (mask >> j & 1) else -a[i][j]
            p *= f
        total += -p if (bin(mask).count("1") & 1) else p
    return total


def per_nw(A) -> int:
    """per(A) from the doubled Nijenhuis-Wilf sum: (-1)^{n-1} V / 2^{n-1}, checking divisibility."""
    a = _as_lists(A)
    n = len(a)
    if n == 0:
        return 1
    V = nw_doubled_sum(a)
    if n % 2 == 0:
        V = -V
    q, r = divmod(V, 1 << (n - 1))
    if r:
        raise ArithmeticError("doubled NW sum is not divisible by 2^(n-1)")
    return q


# --------------------------------------------------------------------------- eq. (2)
def _transpose(a):
    return [list(c) for c in zip(*a)] if a else []


def choose_line(A) -> tuple[str, int, int]:
    """Step 1 of Algorithm H_per: the minimal number s of nonzeros in one row or column.

    Returns (kind, index, s) with kind 'row' or 'col'. Ties (the paper leaves them open)
    go to rows before columns, then to the lowest index."""
    a = _as_lists(A)
    n = len(a)
    best = None
    for i in range(n):
        k = sum(1 for x in a[i] if x != 0)
        if best is None or k < best[2]:
            best = ("row", i, k)
    for j in range(n):
        k = sum(1 for i in range(n) if a[i][j] != 0)
        if k < best[2]:
            best = ("col", j, k)
    return best


def e2_children(A, kind: str = "row", index: int = 0) -> list[list[list[int]]]:
    """One application of expansion (2) (Section 2.1) along one row (or column).

    For a row whose first entries are a, b, c, d (in column order) with columns y1..y4 below
    them and the rest x^T:
        per(A) = per([a*y2 + b*y1, y3, y4, Z]) + per([y1, y2, c*y4 + d*y3, Z]) + per(A3),
    where the row itself is deleted in the first two terms and A3 is A with a, b, c, d set
    to zero. Here a..d are the row's nonzeros in increasing column order; when the row has
    an odd number of them, the missing partner is a zero entry in the lowest-index column
    that is zero in this row, or the lowest other column if the row has no zero (the
    partner's coefficient is 0, which turns the merge into "delete the column of the
    nonzero and scale the partner column by it"). A3 is expanded again the same way
    until the row is exhausted, so a row with k nonzeros gives ceil(k/2) children of order
    n-1; a child with a zero column (every pair has coefficient 0) is still returned.

    A column is expanded by applying the same rule to the transpose (per(A^T) = per(A)).
    Returns the list of children as lists of lists."""
    a = _as_lists(A)
    if kind == "col":
        a = _transpose(a)
    elif kind != "row":
        raise ValueError(kind)
    n = len(a)
    r = index
    nz = [j for j in range(n) if a[r][j] != 0]
    zero_cols = [j for j in range(n) if a[r][j] == 0]
    children = []
    for t in range(0, len(nz), 2):
        p = nz[t]
        if t + 1 < len(nz):
            q = nz[t + 1]
            ca, cb = a[r][p], a[r][q]
        else:
            # odd last nonzero: its partner carries coefficient 0 (a zero entry of the row
            # if there is one, else the lowest other column), which leaves the Laplace term
            # a[r][p] * per(minor without row r and column p) with column q scaled by a[r][p]
            q = zero_cols[0] if zero_cols else min(j for j in range(n) if j != p)
            ca, cb = a[r][p], 0
        # positions p (coefficient a, column y1) and q (coefficient b, column y2):
        # the merged column a*y2 + b*y1 replaces the pair; it is placed at min(p, q).
        keep, drop = min(p, q), max(p, q)
        child = []
        for i in range(n):
            if i == r:
                continue
            row = []
            for j in range(n):
                if j == drop:
                    continue
                if j == keep:
                    row.append(ca * a[i][q] + cb * a[i][p])
                else:
                    row.append(a[i][j])
            child.append(row)
        if kind == "col":
            child = _transpose(child)
        children.append(child)
    return children


def per_hybrid(A, leaf=None) -> int:
    """Algorithm H_per (Section 2.1): with s the minimal nonzero count of a row or column,
    if n > 2 and s < 5 split by expansion (2) and sum the children, else evaluate by R-NW.

    ``leaf`` evaluates the R-NW case (default: Ryser's formula). Orders 0, 1 and 2 are
    evaluated directly (the empty product is 1)."""
    leaf = leaf or per_ryser
    a = _as_lists(A)
    n = len(a)
    if n == 0:
        return 1
    if n == 1:
        return a[0][0]
    if n == 2:
        return a[0][0] * a[1][1] + a[0][1] * a[1][0]
    kind, idx, s = choose_line(a)
    if s == 0:
        return 0
    if s < 5:
        return sum(per_hybrid(c, leaf) for c in e2_children(a, kind, idx))
    return leaf(a)


# --------------------------------------------------------------------------- frontier DP
def _open_cost(supp, order) -> int:
    """sum over steps of 2^(number of open columns): a bound on the DP's work for this order."""
    last = {}
    for pos, i in enumerate(order):
        for j in supp[i]:
            last[j] = pos
    opened: set[int] = set()
    cost = 0
    for pos, i in enumerate(order):
        opened |= supp[i]
        opened = {j for j in opened if last[j] > pos}
        cost += 1 << len(opened)
    return cost


def _row_order(a) -> list[int]:
    """A row order that keeps the set of open columns small (any order gives the same result).

    Candidates: breadth-first orders of the row graph (rows joined when they share a
    column) from every start row; the one with the smallest open-column cost is used."""
    n = len(a)
    supp = [frozenset(j for j in range(n) if a[i][j]) for i in range(n)]
    col_rows = [[i for i in range(n) if a[i][j]] for j in range(n)]
    nbr = [sorted({r for j in supp[i] for r in col_rows[j]} - {i}) for i in range(n)]
    best = None
    for s in range(n):
        seen = [False] * n
        order = []
        for root in [s] + list(range(n)):
            if seen[root]:
                continue
            seen[root] = True
            q = [root]
            while q:
                u = q.pop(0)
                order.append(u)
                for w in nbr[u]:
                    if not seen[w]:
                        seen[w] = True
                        q.append(w)
        c = _open_cost(supp, order)
        if best is None or c < best[0]:
            best = (c, order)
    return best[1]


def per_dp(A) -> int:
    """Permanent by a dynamic programme over rows (an independent textbook route, not the paper's).

    Rows are taken in a fixed order. A state records which of the currently open columns
    (touched by a processed row and still touched by an unprocessed one) are already
    matched; its weight is the sum, over partial assignments of the processed rows to
    distinct columns, of the product of the chosen entries. A column whose last row has
    been processed must be matched, else the state is dropped. After the last row every
    column is closed and the weight of the empty state is per(A)."""
    a = _as_lists(A)
    n = len(a)
    if n == 0:
        return 1
    for j in range(n):
        if not any(a[i][j] for i in range(n)):
            return 0
    order = _row_order(a)
    last = {}
    for pos, i in enumerate(order):
        for j in range(n):
            if a[i][j]:
                last[j] = pos
    states: dict[int, int] = {0: 1}
    for pos, i in enumerate(order):
        nz = [(j, a[i][j]) for j in range(n) if a[i][j]]
        new: dict[int, int] = defaultdict(int)
        for mask, w in states.items():
            for j, v in nz:
                bit = 1 << j
                if not mask & bit:
                    new[mask | bit] += w * v
        closing = [j for j, _ in nz if last[j] == pos]
        for j in closing:
            bit = 1 << j
            new = {m ^ bit: w for m, w in new.items() if m & bit}
        states = dict(new)
        if not states:
            return 0
    return states.get(0, 0)


def per_auto(A) -> int:
    """Exact per(A) by the cheapest applicable route: brute force for n <= 6, else the DP."""
    a = _as_lists(A)
    return per_brute(a) if len(a) <= 6 else per_dp(a)


# --------------------------------------------------------------------------- jobs of PH
def expand_leaves(A, m_cut: int, s_leaf: int = 5, m_cap: int = 40,
                  limit: int | None = None) -> list[list[list[int]]]:
    """The sub-matrix jobs of a pre-expansion (Algorithm PH, Step 2) with a size-based stop.

    Depth-first over the expansion tree, children in pair order: a node whose smallest
    line has s = 0 nonzeros is dropped (per = 0); it is a job when its order is at most
    m_cut (or at most 2), or when s >= s_leaf and its order is at most m_cap (Algorithm
    H_per hands such a node to R-NW); otherwise it is split by expansion (2) along that
    line (see ``choose_line`` and ``e2_children``). Returns the jobs in depth-first order;
    by Step 4 of Algorithm PH their permanents sum to per(A). With ``limit`` only the first
    ``limit`` jobs are produced."""
    out = []

    def rec(a):
        if limit is not None and len(out) >= limit:
            return
        n = len(a)
        if n == 0:
            out.append(a)
            return
        kind, idx, s = choose_line(a)
        if s == 0:
            return
        if n <= m_cut or n <= 2 or (s >= s_leaf and n <= m_cap):
            out.append(a)
            return
        for c in e2_children(a, kind, idx):
            rec(c)

    rec(_as_lists(A))
    return out
