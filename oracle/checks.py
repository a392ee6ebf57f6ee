"""Result validators -- TEST INFRASTRUCTURE ONLY.

* ``check_parents``: the Graph500-style parent check.  Several parent trees are
  correct (the cascade's ANY reduction picks any one of the duplicate sources,
  Cascade 1, Eq. advance), so parents are validated, not compared: the source
  is its own parent at depth 0, every other reached vertex has a parent one
  level up joined to it by a CSR edge, unreached vertices have parent -1.
* ``check_levels``: invariants of exact BFS depths that hold at any size:
  depth 0 only at the source; no edge (u,v) with u reached has v unreached or
  depth(v) > depth(u)+1; every reached v other than the source has an
  in-neighbour at depth(v)-1.
* ``frontiers_from_levels``: F_k, P_k read off the depths, with the identity
  F_k = P_k and not P_{k-1} (Table 3, variant 26).
"""
from __future__ import annotations

import numpy as np


def _edges(row_ptr, col_idx):
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    src = np.repeat(np.arange(len(row_ptr) - 1, dtype=np.int64), np.diff(row_ptr))
    return src, np.asarray(col_idx, dtype=np.int64)


def check_levels(row_ptr, col_idx, source: int, levels) -> str | None:
    """Returns None when the invariants hold, else a message."""
    lv = np.asarray(levels, dtype=np.int64)
    n = len(row_ptr) - 1
    if lv.shape[0] != n:
        return "levels has wrong length"
    if lv[source] != 0:
        return "source depth is not 0"
    if ((lv == 0).sum()) != 1:
        return "depth 0 at a vertex other than the source"
    if (lv < -1).any():
        return "depth below -1"
    s, d = _edges(row_ptr, col_idx)
    ls, ld = lv[s], lv[d]
    reached_src = ls >= 0
    if (reached_src & (ld < 0)).any():
        return "edge from a reached vertex to an unreached one"
    if (reached_src & (ld > ls + 1)).any():
        return "edge (u,v) with depth(v) > depth(u)+1"
    # every reached v != source has an in-neighbour one level up
    good = np.zeros(n, dtype=bool)
    ok = reached_src & (ld == ls + 1)
    good[d[ok]] = True
    need = (lv > 0)
    if (need & ~good).any():
        return "reached vertex without an in-neighbour one level up"
    return None


def edge_keys(row_ptr, col_idx):
    """Sorted keys u * n + v of every CSR edge (u, v), for check_parents on
    many searches of one graph."""
    n = len(row_ptr) - 1
    s, d = _edges(row_ptr, col_idx)
    k = s * n + d
    k.sort()
    return k


def check_parents(row_ptr, col_idx, source: int, levels, parents, keys=None) -> str | None:
    """keys: edge_keys(row_ptr, col_idx) when already at hand."""
    lv = np.asarray(levels, dtype=np.int64)
    pa = np.asarray(parents, dtype=np.int64)
    n = len(row_ptr) - 1
    if pa.shape[0] != n:
        return "parents has wrong length"
    if pa[source] != source:
        return "parent of the source is not the source"
    reached = lv >= 0
    if (pa[~reached] != -1).any():
        return "unreached vertex with a parent"
    v = np.nonzero(reached)[0]
    v = v[v != source]
    p = pa[v]
    if ((p < 0) | (p >= n)).any():
        return "parent out of range"
    if (lv[p] != lv[v] - 1).any():
        return "parent not one level up"
    # edge (p, v) must exist: look it up in p's CSR row (rows need not be sorted)
    key_edges = edge_keys(row_ptr, col_idx) if keys is None else keys
    key = p * n + v
    if key.size == 0:
        return None
    pos = np.searchsorted(key_edges, key)
    pos = np.minimum(pos, max(len(key_edges) - 1, 0))
    if len(key_edges) == 0 or (key_edges[pos] != key).any():
        return "parent edge not in the graph"
    return None


def frontiers_from_levels(levels, k: int):
    """(F_k, P_k) as boolean vectors: F_k = {depth = k}, P_k = {0 <= depth <= k}."""
    lv = np.asarray(levels)
    F = lv == k
    P = (lv >= 0) & (lv <= k)
    return F, P
