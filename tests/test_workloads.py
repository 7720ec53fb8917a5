"""Seeded input generators: determinism and the structure the paper's workloads have."""
import numpy as np
import pytest

import workloads as W


def _cycles_of_length(adj, L):
    """Number of simple cycles of length L (each counted once)."""
    n = len(adj)
    count = 0

    def dfs(start, u, depth, seen):
        nonlocal count
        for w in adj[u]:
            if w == start and depth == L:
                count += 1
            elif w > start and w not in seen and depth < L:
                seen.add(w)
                dfs(start, w, depth + 1, seen)
                seen.remove(w)

    for s in range(n):
        dfs(s, s, 1, {s})
    return count // 2


@pytest.mark.parametrize("n,d,g", [(24, 3, 3), (60, 3, 5), (30, 4, 3)])
def test_regular_graph_is_simple_regular_seeded(n, d, g):
    a1 = W.random_regular_graph(n, d, 5, g)
    a2 = W.random_regular_graph(n, d, 5, g)
    assert a1 == a2
    for u, nb in enumerate(a1):
        assert len(nb) == d and len(set(nb)) == d and u not in nb
        assert all(u in a1[w] for w in nb)
    assert W._girth(a1, 99) >= g


def test_truncated_icosahedron_structure():
    adj = W.truncated_icosahedron()
    assert len(adj) == 60 and all(len(nb) == 3 for nb in adj)
    assert W._girth(adj, 99) == 5
    assert _cycles_of_length(adj, 5) == 12 and _cycles_of_length(adj, 6) == 20


def test_appendix_graphs_are_fullerenes():
    for name, n, hexes in (("c100", 100, 40), ("c60", 60, 20)):
        adj = W.read_appendix_adjacency(name)
        assert len(adj) == n and all(len(nb) == 3 for nb in adj)
        assert all(u in adj[w] for u, nb in enumerate(adj) for w in nb)
        assert _cycles_of_length(adj, 5) == 12 and _cycles_of_length(adj, 6) == hexes


def test_csr_roundtrip():
    A = W.permutation_union_matrix(17, 3, 1)
    rp, ci, v = W.to_csr(A)
    B = np.zeros_like(A)
    for i in range(17):
        B[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
        assert list(ci[rp[i]:rp[i + 1]]) == sorted(ci[rp[i]:rp[i + 1]])
    assert (A == B).all()


def test_serving_mix_is_seeded():
    r1 = W.serving_requests(9, 3)
    r2 = W.serving_requests(9, 3)
    assert [k for k, _ in r1] == [k for k, _ in r2]
    assert all((a == b).all() for (_, a), (_, b) in zip(r1, r2))
    assert all(30 <= A.shape[0] <= 101 for _, A in r1)
