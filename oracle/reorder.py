"""Degree renumbering of a graph -- TEST INFRASTRUCTURE ONLY (see the package
docstring for who may import it).

The paper renumbers every graph before it times a search (reverse
Cuthill-McKee, Sec. "Experiment Setup", preprocessing paragraph).  The
library's preprocessing step uses another order, which this module defines
plainly:

  * new id i is the vertex with the i-th largest out-degree; vertices of
    equal out-degree keep their relative order (increasing old id);
  * the renumbered graph has the edge (new u, new v) for every edge (u, v),
    with every adjacency row in increasing order.

A search does not depend on the numbering: depth_new[new(v)] = depth_old[v]
from new(s) and s.  The tests pin this module with a hand-worked example,
invariants of the order and that identity on brute-force distances.
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
