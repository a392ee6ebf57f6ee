"""Vertex renumberings of a graph (by degree; reverse Cuthill-McKee) -- TEST
INFRASTRUCTURE ONLY (see the package docstring for who may import it).

The paper renumbers every graph before it times a search (reverse
Cuthill-McKee, Sec. "Experiment Setup", preprocessing paragraph).  The
library offers that order and one by degree; this module defines both
plainly:

  * degree_order: new id i is the vertex with the i-th largest out-degree;
    vertices of equal out-degree keep their relative order (increasing old id);
  * rcm_order: reverse Cuthill-McKee with the rules in its docstring;
  * renumber: the renumbered graph has the edge (new u, new v) for every edge
    (u, v), with every adjacency row in increasing order.

A search does not depend on the numbering: depth_new[new(v)] = depth_old[v]
from new(s) and s.  The tests pin this module with hand-worked examples,
invariants of the orders and that identity on brute-force distances.
"""
from __future__ import annotations

import numpy as np


def degree_order(row_ptr):
    """(new_of_old, old_of_new) int32: a stable sort of the vertices by
    decreasing out-degree."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    old_of_new = np.argsort(-deg, kind="stable").astype(np.int32)
    new_of_old = np.empty_like(old_of_new)
    new_of_old[old_of_new] = np.arange(old_of_new.size, dtype=np.int32)
    return new_of_old, old_of_new


def renumber(row_ptr, col_idx, new_of_old):
    """The adjacency (row_ptr, col_idx) with every vertex id v replaced by
    new_of_old[v]; rows ascending.  Returns int32 (row_ptr, col_idx)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    new_of_old = np.asarray(new_of_old, dtype=np.int64)
    n = row_ptr.size - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    nsrc, ndst = new_of_old[src], new_of_old[col_idx]
    order = np.lexsort((ndst, nsrc))  # by new source, then new destination
    counts = np.bincount(nsrc, minlength=n)
    out_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=out_ptr[1:])
    return out_ptr.astype(np.int32), ndst[order].astype(np.int32)


def rcm_order(row_ptr, col_idx, csc_ptr=None, csc_idx=None):
    """(new_of_old, old_of_new) of reverse Cuthill-McKee, as this library
    defines it (the paper names the method, not its details):

      * neighbours of v: its out-neighbours, and for a directed graph given with
        its transpose also its in-neighbours (the undirected structure);
        deg(v) = the length of that list (duplicates and self-loops counted);
      * vertices are taken in the order (deg, id);
      * Cuthill-McKee: while vertices remain, start at the remaining vertex
        that is first in that order; visit breadth-first, appending each
        visited vertex's unvisited neighbours in that order;
      * reverse: new id i is the (n-1-i)-th vertex of the Cuthill-McKee order.
    Plain Python loops: small graphs only."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    n = row_ptr.size - 1
    rows = [list(col_idx[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]
    if csc_ptr is not None:
        csc_ptr = np.asarray(csc_ptr, dtype=np.int64)
        csc_idx = np.asarray(csc_idx, dtype=np.int64)
        for v in range(n):
            rows[v] += list(csc_idx[csc_ptr[v]:csc_ptr[v + 1]])
    deg = [len(r) for r in rows]
    rank_key = sorted(range(n), key=lambda v: (deg[v], v))
    visited = [False] * n
    order = []
    for s in rank_key:  # the remaining vertex first in (deg, id) order
        if visited[s]:
            continue
        visited[s] = True
        order.append(s)
        head = len(order) - 1
        while head < len(order):
            u = order[head]
            head += 1
            fresh = sorted({w for w in rows[u] if not visited[w]}, key=lambda w: (deg[w], w))
            for w in fresh:
                visited[w] = True
                order.append(w)
    old_of_new = np.array(order[::-1], dtype=np.int32)
    new_of_old = np.empty(n, dtype=np.int32)
    new_of_old[old_of_new] = np.arange(n, dtype=np.int32)
    return new_of_old, old_of_new
