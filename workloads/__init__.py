"""Seeded synthetic inputs for the sparse-permanent path.

This module only builds input matrices (graphs, adjacency and small-integer sparse
matrices) and reads the paper's appendix adjacency lists. It holds none of the
permanent arithmetic, so both the CPU oracle's tests and the GPU path's tests, the
smoke check and the benchmark can draw from it.

Every generator takes an explicit seed and uses ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import os
from collections import deque

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "tests", "golden")


# --------------------------------------------------------------------------- graphs
def _girth(adj: list[list[int]], cap: int) -> int:
    """Length of the shortest cycle, or ``cap`` if it is at least ``cap`` (BFS per vertex)."""
    n = len(adj)
    best = cap
    for s in range(n):
        dist = [-1] * n
        parent = [-1] * n
        dist[s] = 0
        q = deque([s])
        while q:
            u = q.popleft()
            if 2 * dist[u] + 1 >= best:
                break
            for w in adj[u]:
                if dist[w] < 0:
                    dist[w] = dist[u] + 1
                    parent[w] = u
                    q.append(w)
                elif parent[u] != w:
                    best = min(best, dist[u] + dist[w] + 1)
    return best


def random_regular_graph(n: int, d: int, seed: int, min_girth: int = 3,
                         max_tries: int = 200000) -> list[list[int]]:
    """Random simple d-regular graph on n vertices by the configuration model.

    The n*d half-edges ("points") are shuffled and consecutive pairs become edges.
    Draws with a loop or a repeated edge are rejected, and so are draws whose girth
    is below ``min_girth``. Returns sorted 0-based neighbour lists.
    """
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    rng = np.random.default_rng(seed)
    pts = np.repeat(np.arange(n), d)
    for _ in range(max_tries):
        perm = rng.permutation(pts)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        keys = lo.astype(np.int64) * n + hi
        if np.unique(keys).size != keys.size:
            continue
        adj = [[] for _ in range(n)]
        for u, v in zip(a.tolist(), b.tolist()):
            adj[u].append(v)
            adj[v].append(u)
        adj = [sorted(x) for x in adj]
        if min_girth > 3 and _girth(adj, min_girth) < min_girth:
            continue
        return adj
    raise RuntimeError("configuration model: no simple graph found")


def icosahedron() -> list[list[int]]:
    """The icosahedron: vertices (0,+-1,+-phi) and cyclic shifts; edges join points at distance 2."""
    phi = (1 + 5 ** 0.5) / 2
    pts = []
    for s1 in (1, -1):
        for s2 in (1, -1):
            base = (0.0, s1 * 1.0, s2 * phi)
            for r in range(3):
                pts.append(tuple(base[(i - r) % 3] for i in range(3)))
    P = np.array(pts)
    D = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=-1)
    return [sorted(int(j) for j in np.nonzero(np.abs(D[i] - 2.0) < 1e-9)[0]) for i in range(12)]


def truncated_icosahedron() -> list[list[int]]:
    """The truncated icosahedron (C60 cage) built from the icosahedron.

    Each directed icosahedron edge u->v becomes a vertex. It is joined to v->u (the edge
    between two hexagons) and to u->w for the two neighbours w of u that are adjacent to v
    (the pentagon around u). Gives 60 vertices, 3-regular, 12 pentagons and 20 hexagons.
    """
    ico = icosahedron()
    darts = [(u, v) for u in range(12) for v in ico[u]]
    idx = {dv: i for i, dv in enumerate(darts)}
    adj = [[] for _ in darts]
    for (u, v), i in idx.items():
        adj[i].append(idx[(v, u)])
        for w in ico[u]:
            if w != v and w in ico[v]:
                adj[i].append(idx[(u, w)])
    return [sorted(x) for x in adj]


def read_appendix_adjacency(name: str) -> list[list[int]]:
    """0-based neighbour lists of ``c100`` or ``c60`` from the paper's appendix fixtures."""
    path = os.path.join(GOLDEN_DIR, f"{name}_adjacency.txt")
    adj = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            adj.append(sorted(int(x) - 1 for x in line.split()))
    return adj


def read_c100_subpermanents() -> tuple[int, dict[int, int]]:
    """(printed total, {No.: per}) of the paper's appendix table for C100."""
    path = os.path.join(GOLDEN_DIR, "c100_t12_subpermanents.txt")
    total, vals = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split()
            if a == "TOTAL":
                total = int(b)
            else:
                vals[int(a)] = int(b)
    return total, vals


# --------------------------------------------------------------------------- matrices
def adjacency_matrix(adj: list[list[int]]) -> np.ndarray:
    """Dense 0-1 uint32 adjacency matrix of a neighbour-list graph."""
    n = len(adj)
    A = np.zeros((n, n), dtype=np.uint32)
    for i, nb in enumerate(adj):
        A[i, nb] = 1
    return A


def random_cubic_matrix(n: int, seed: int, min_girth: int = 3) -> np.ndarray:
    return adjacency_matrix(random_regular_graph(n, 3, seed, min_girth))


def random_quartic_matrix(n: int, seed: int, min_girth: int = 3) -> np.ndarray:
    return adjacency_matrix(random_regular_graph(n, 4, seed, min_girth))


def permutation_union_matrix(n: int, k: int, seed: int, lo: int = 1, hi: int = 4) -> np.ndarray:
    """Sparse non-negative integer matrix: the union of k random permutation patterns, values U{lo..hi}.

    Collisions between permutations merge into one entry, so rows have at most k nonzeros
    and the permanent is at least 1 (each permutation is a positive diagonal).
    """
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.uint32)
    for _ in range(k):
        p = rng.permutation(n)
        A[np.arange(n), p] = rng.integers(lo, hi + 1, size=n, dtype=np.int64).astype(np.uint32)
    return A


def random_sparse_int_matrix(n: int, density_per_row: int, seed: int, lo: int = 0,
                             hi: int = 8) -> np.ndarray:
    """n x n matrix with ``density_per_row`` random positions per row, values U{lo..hi} (zeros allowed)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.uint32)
    for i in range(n):
        cols = rng.choice(n, size=min(density_per_row, n), replace=False)
        A[i, cols] = rng.integers(lo, hi + 1, size=cols.size, dtype=np.int64).astype(np.uint32)
    return A


def random_01_matrix(n: int, nnz: int, seed: int) -> np.ndarray:
    """n x n 0-1 matrix with ``nnz`` ones at uniformly random distinct positions (the random
    matrices of a given size and sparsity of the regression study; zero lines allowed)."""
    rng = np.random.default_rng(seed)
    A = np.zeros(n * n, dtype=np.uint32)
    A[rng.choice(n * n, size=min(nnz, n * n), replace=False)] = 1
    return A.reshape(n, n)


def to_csr(A: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(row_ptr int32[n+1], col_idx int32[nnz], val uint32[nnz]) with sorted columns per row."""
    A = np.asarray(A)
    n = A.shape[0]
    rows, cols = np.nonzero(A)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, cols.astype(np.int32), A[rows, cols].astype(np.uint32)


# --------------------------------------------------------------------------- workloads
def config_n24(seeds=range(10)) -> list[np.ndarray]:
    """Random 3-regular simple graphs on 24 vertices (adjacency 0-1), one per seed."""
    return [random_cubic_matrix(24, s) for s in seeds]


def config_n60(n_random: int = 16) -> list[tuple[str, np.ndarray]]:
    """The truncated icosahedron plus ``n_random`` random cubic girth>=5 graphs on 60 vertices."""
    out = [("truncated_icosahedron", adjacency_matrix(truncated_icosahedron()))]
    for s in range(n_random):
        out.append((f"cubic60_g5_seed{s}", random_cubic_matrix(60, s, min_girth=5)))
    return out


def config_n80(n_graphs: int = 8) -> list[tuple[str, np.ndarray]]:
    """Random cubic girth>=5 graphs on 80 vertices, seeds 0..n_graphs-1."""
    return [(f"cubic80_g5_seed{s}", random_cubic_matrix(80, s, min_girth=5)) for s in range(n_graphs)]


def poisson_arrivals(n_requests: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: cumulative seeded exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n_requests))


def serving_requests(n_requests: int, seed: int, n_lo: int = 30, n_hi: int = 100) -> list[tuple[str, np.ndarray]]:
    """Mixed request stream: n ~ U{n_lo..n_hi}; a third each of 3-regular 0-1, 4-regular 0-1 and
    small-integer (values 1..4) sparse matrices built from three random permutations."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_requests):
        kind = r % 3
        n = int(rng.integers(n_lo, n_hi + 1))
        s = int(rng.integers(0, 2 ** 31 - 1))
        if kind == 0:
            n += n % 2
            out.append((f"cubic{n}", random_cubic_matrix(n, s)))
        elif kind == 1:
            out.append((f"quartic{n}", random_quartic_matrix(n, s)))
        else:
            out.append((f"int3perm{n}", permutation_union_matrix(n, 3, s, 1, 4)))
    return out
