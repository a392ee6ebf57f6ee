"""Brute-force unit-weight distances -- TEST INFRASTRUCTURE ONLY.

Floyd-Warshall over the 0/1 adjacency matrix: the depth the paper defines
(minimum number of hops from the query vertex, Sec. "Expressing BFS with
EDGE") is the all-pairs shortest-path distance with every edge weighted 1.
This is a different algorithm from the queue BFS it pins, O(n^3), so it is
used on tiny graphs only.
"""
from __future__ import annotations

import numpy as np

INF = np.iinfo(np.int64).max // 4


def all_pairs_hops(n: int, edges) -> np.ndarray:
    """dist[s, d] = fewest directed edges from s to d (INF when unreachable)."""
    D = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for s, d in edges:
        if s != d:
            D[s, d] = 1
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def levels_from(n: int, edges, source: int) -> np.ndarray:
    """Depth of every vertex from ``source`` as int32, -1 when unreachable."""
    D = all_pairs_hops(n, edges)
    row = D[source]
    return np.where(row >= INF, -1, row).astype(np.int32)


def edges_of_csr(row_ptr, col_idx):
    row_ptr = np.asarray(row_ptr)
    out = []
    for u in range(len(row_ptr) - 1):
        for j in range(row_ptr[u], row_ptr[u + 1]):
            out.append((u, int(col_idx[j])))
    return out
