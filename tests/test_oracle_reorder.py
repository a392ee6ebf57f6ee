"""Pins of the oracle's degree renumbering (oracle/reorder.py):

* a hand-worked example, order and renumbered CSR written out by hand;
* invariants on random graphs: a bijection, out-degrees non-increasing in new
  order with ties in increasing old id, the edge set carried over exactly,
  rows ascending;
* numbering does not change distances: brute-force hop counts on the
  renumbered graph from new(s) equal those on the original from s, moved to
  the new ids;
* planted mistakes (a swapped pair in the order, an unsorted row) fail the
  invariant checks.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import graphgen as gg
from oracle import brute, reorder


def test_hand_example():
    # out-degrees 0:1 1:0 2:3 3:0 4:2 -> order 2, 4, 0, then the ties 1, 3
    g = gg.from_edge_list(5, [(0, 1), (2, 0), (2, 1), (2, 3), (4, 2), (4, 3)], False)
    new_of_old, old_of_new = reorder.degree_order(g.row_ptr)
    assert list(old_of_new) == [2, 4, 0, 1, 3]
    assert list(new_of_old) == [2, 3, 0, 4, 1]
    rp, ci = reorder.renumber(g.row_ptr, g.col_idx, new_of_old)
    # (0,1)->(2,3) (2,0)->(0,2) (2,1)->(0,3) (2,3)->(0,4) (4,2)->(1,0) (4,3)->(1,4)
    assert list(rp) == [0, 3, 5, 6, 6, 6]
    assert list(ci) == [2, 3, 4, 0, 4, 3]


def order_problems(row_ptr, new_of_old, old_of_new):
    n = len(row_ptr) - 1
    if sorted(old_of_new.tolist()) != list(range(n)):
        return "not a permutation"
    if not np.array_equal(new_of_old[old_of_new], np.arange(n)):
        return "maps are not inverse"
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))[old_of_new]
    if np.any(np.diff(deg) > 0):
        return "out-degree increases"
    tie = np.diff(deg) == 0
    if np.any(np.diff(old_of_new.astype(np.int64))[tie] < 0):
        return "tie out of id order"
    return None


def graph_problems(row_ptr, col_idx, rp, ci, new_of_old):
    if np.any(np.diff(rp) < 0) or rp[0] != 0 or rp[-1] != len(ci):
        return "bad offsets"
    for i in range(len(rp) - 1):
        if np.any(np.diff(ci[rp[i]:rp[i + 1]]) < 0):
            return f"row {i} not ascending"
    old = sorted((int(new_of_old[u]), int(new_of_old[v])) for u, v in brute.edges_of_csr(row_ptr, col_idx))
    new = sorted(brute.edges_of_csr(rp, ci))
    return None if old == new else "edge set differs"


@st.composite
def tiny_graphs(draw):
    n = draw(st.integers(1, 30))
    m = draw(st.integers(0, 4 * n))
    edges = [(draw(st.integers(0, n - 1)), draw(st.integers(0, n - 1))) for _ in range(m)]
    return n, edges, draw(st.booleans()), draw(st.integers(0, n - 1))


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_graphs())
def test_invariants_and_distances(case):
    n, edges, symmetric, s = case
    g = gg.from_edge_list(n, edges, symmetric)
    new_of_old, old_of_new = reorder.degree_order(g.row_ptr)
    assert order_problems(g.row_ptr, new_of_old, old_of_new) is None
    rp, ci = reorder.renumber(g.row_ptr, g.col_idx, new_of_old)
    assert graph_problems(g.row_ptr, g.col_idx, rp, ci, new_of_old) is None
    d_old = brute.levels_from(n, brute.edges_of_csr(g.row_ptr, g.col_idx), s)
    d_new = brute.levels_from(n, brute.edges_of_csr(rp, ci), int(new_of_old[s]))
    np.testing.assert_array_equal(d_new[new_of_old], d_old)


def test_rmat_invariants():
    g = gg.rmat(10, seed=31)
    new_of_old, old_of_new = reorder.degree_order(g.row_ptr)
    assert order_problems(g.row_ptr, new_of_old, old_of_new) is None
    rp, ci = reorder.renumber(g.row_ptr, g.col_idx, new_of_old)
    assert graph_problems(g.row_ptr, g.col_idx, rp, ci, new_of_old) is None


def test_planted_mistakes_fail():
    g = gg.rmat(8, seed=5)
    new_of_old, old_of_new = reorder.degree_order(g.row_ptr)
    bad = old_of_new.copy()
    bad[[0, -1]] = bad[[-1, 0]]  # a leaf first, a hub last
    inv = np.empty_like(bad)
    inv[bad] = np.arange(bad.size)
    assert order_problems(g.row_ptr, inv, bad) is not None
    rp, ci = reorder.renumber(g.row_ptr, g.col_idx, new_of_old)
    ci2 = ci.copy()
    r0 = int(np.argmax(np.diff(rp)))
    ci2[rp[r0]:rp[r0 + 1]] = ci2[rp[r0]:rp[r0 + 1]][::-1]  # a row reversed
    assert graph_problems(g.row_ptr, g.col_idx, rp, ci2, new_of_old) is not None
    ci3 = ci.copy()
    ci3[0] = (ci3[0] + 1) % g.n  # one edge moved
    assert graph_problems(g.row_ptr, g.col_idx, rp, ci3, new_of_old) is not None
