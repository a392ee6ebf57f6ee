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


# ---------------------------------------------------------------- RCM
def test_rcm_hand_example():
    # component A: 0-1, 0-2, 0-3, 3-4, 4-5; component B: 6-7; 8 isolated.
    # degrees 0:3 1:1 2:1 3:2 4:2 5:1 6:1 7:1 8:0; (deg, id) order: 8 1 2 5 6 7 3 4 0.
    # Cuthill-McKee: start 8; then 1 -> 0 -> {2 (deg 1), 3 (deg 2)} -> 4 -> 5; then 6 -> 7
    #   = 8 1 0 2 3 4 5 6 7, reversed for new ids 0..8.
    g = gg.from_edge_list(9, [(0, 1), (0, 2), (0, 3), (3, 4), (4, 5), (6, 7)], True)
    new_of_old, old_of_new = reorder.rcm_order(g.row_ptr, g.col_idx)
    assert list(old_of_new) == [7, 6, 5, 4, 3, 2, 0, 1, 8]
    assert list(new_of_old) == [6, 7, 5, 4, 3, 2, 1, 0, 8]


def test_rcm_directed_uses_both_directions():
    # 0 -> 1 -> 2 only as out-edges: with the transpose the structure is the path 0-1-2,
    # degrees 1, 2, 1: start 0, then 1, then 2; reversed: 2 1 0
    g = gg.from_edge_list(3, [(0, 1), (1, 2)], False).with_csc()
    _, old_of_new = reorder.rcm_order(g.row_ptr, g.col_idx, g.csc_ptr, g.csc_idx)
    assert list(old_of_new) == [2, 1, 0]
    # out-edges alone: vertex 2 has degree 0 and comes first in Cuthill-McKee order
    _, o2 = reorder.rcm_order(g.row_ptr, g.col_idx)
    assert o2[-1] == 2


def cm_problems(row_ptr, col_idx, old_of_new):
    """Checks the reversed order against what Cuthill-McKee fixes: components
    are contiguous, each starts at its first vertex in (deg, id) order, and
    inside a component the hop distance from its start never decreases."""
    n = len(row_ptr) - 1
    cm = list(old_of_new[::-1])
    edges = brute.edges_of_csr(row_ptr, col_idx)
    deg = np.diff(np.asarray(row_ptr))
    i = 0
    seen = set()
    while i < n:
        s = cm[i]
        remaining = [v for v in range(n) if v not in seen]
        first = min(remaining, key=lambda v: (deg[v], v))
        if s != first:
            return f"component at {i} starts at {s}, not {first}"
        dist = brute.levels_from(n, edges, s)
        comp = [v for v in range(n) if dist[v] >= 0]
        block = cm[i:i + len(comp)]
        if sorted(block) != sorted(comp):
            return f"component of {s} not contiguous"
        if any(dist[block[j]] > dist[block[j + 1]] for j in range(len(block) - 1)):
            return f"component of {s} not in breadth-first order"
        seen.update(comp)
        i += len(comp)
    return None


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_graphs())
def test_rcm_invariants_and_distances(case):
    n, edges, _, s = case
    g = gg.from_edge_list(n, edges, True)
    new_of_old, old_of_new = reorder.rcm_order(g.row_ptr, g.col_idx)
    assert sorted(old_of_new.tolist()) == list(range(n))
    assert np.array_equal(new_of_old[old_of_new], np.arange(n))
    assert cm_problems(g.row_ptr, g.col_idx, old_of_new) is None
    rp, ci = reorder.renumber(g.row_ptr, g.col_idx, new_of_old)
    d_old = brute.levels_from(n, brute.edges_of_csr(g.row_ptr, g.col_idx), s)
    d_new = brute.levels_from(n, brute.edges_of_csr(rp, ci), int(new_of_old[s]))
    np.testing.assert_array_equal(d_new[new_of_old], d_old)


def _bandwidth(row_ptr, col_idx):
    src = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    return int(np.abs(src - np.asarray(col_idx)).max()) if len(col_idx) else 0


def test_rcm_bandwidth_of_shuffled_path_and_grid():
    rng = np.random.default_rng(3)
    n = 200
    lab = rng.permutation(n)
    g = gg.from_edge_list(n, [(int(lab[i]), int(lab[i + 1])) for i in range(n - 1)], True)
    n2o, _ = reorder.rcm_order(g.row_ptr, g.col_idx)
    assert _bandwidth(*reorder.renumber(g.row_ptr, g.col_idx, n2o)) == 1
    side = 12
    lab = rng.permutation(side * side)
    e = [(int(lab[r * side + c]), int(lab[r * side + c + 1])) for r in range(side) for c in range(side - 1)]
    e += [(int(lab[r * side + c]), int(lab[(r + 1) * side + c])) for r in range(side - 1) for c in range(side)]
    g = gg.from_edge_list(side * side, e, True)
    assert _bandwidth(g.row_ptr, g.col_idx) > 4 * side  # the shuffled labels
    n2o, _ = reorder.rcm_order(g.row_ptr, g.col_idx)
    # breadth-first from a corner: levels are anti-diagonals of at most `side` vertices
    assert _bandwidth(*reorder.renumber(g.row_ptr, g.col_idx, n2o)) <= 2 * side


def test_rcm_planted_mistake_fails():
    g = gg.from_edge_list(9, [(0, 1), (0, 2), (0, 3), (3, 4), (4, 5), (6, 7)], True)
    _, old_of_new = reorder.rcm_order(g.row_ptr, g.col_idx)
    bad = old_of_new.copy()
    bad[[2, 3]] = bad[[3, 2]]  # two vertices of different depth swapped
    assert cm_problems(g.row_ptr, g.col_idx, bad) is not None
