"""Pins of the CPU oracle against facts fixed independently of it.

* brute force: Floyd-Warshall all-pairs hop counts on random tiny graphs
  (directed and undirected, with self-loops, duplicate edges, isolated vertices
  and several components);
* closed forms: path, cycle, star, complete graph, binary tree, full grid
  (Manhattan distance, also at 4096 x 4096);
* invariants of exact depths and Graph500-style parents on R-MAT and directed
  graphs, and the frontier identity F_k = P_k and not P_{k-1}
  (Table 3, variant 26);
* planted mistakes: the validators reject corrupted depths and parents.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import graphgen as gg
import oracle
from oracle import brute, checks


def _graph(n, edges, symmetric):
    return gg.from_edge_list(n, edges, symmetric)


@st.composite
def tiny_graphs(draw):
    n = draw(st.integers(1, 24))
    m = draw(st.integers(0, 3 * n))
    edges = [(draw(st.integers(0, n - 1)), draw(st.integers(0, n - 1))) for _ in range(m)]
    symmetric = draw(st.booleans())
    s = draw(st.integers(0, n - 1))
    return n, edges, symmetric, s


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_graphs())
def test_oracle_matches_brute_force(case):
    n, edges, symmetric, s = case
    g = _graph(n, edges, symmetric)
    lv, par, nl = oracle.bfs(g.row_ptr, g.col_idx, s)
    all_edges = brute.edges_of_csr(g.row_ptr, g.col_idx)
    ref = brute.levels_from(n, all_edges, s)
    np.testing.assert_array_equal(lv, ref)
    assert nl == int(ref.max()) + 1
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, par) is None
    assert checks.check_levels(g.row_ptr, g.col_idx, s, lv) is None


def test_brute_force_itself_on_hand_graph():
    # 0->1->2->3 plus 0->2: hop counts 0,1,1,2 from 0; 3 unreachable from 1's
    # reverse direction (directed).
    D = brute.all_pairs_hops(4, [(0, 1), (1, 2), (2, 3), (0, 2)])
    assert list(D[0]) == [0, 1, 1, 2]
    assert D[3, 0] >= brute.INF


def _path(n):
    return [(i, i + 1) for i in range(n - 1)]


@pytest.mark.parametrize("n", [1, 2, 17, 1000])
def test_closed_form_path(n):
    g = _graph(n, _path(n), True)
    lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, 0)
    np.testing.assert_array_equal(lv, np.arange(n))


@pytest.mark.parametrize("n", [3, 10, 11, 999])
def test_closed_form_cycle(n):
    g = _graph(n, _path(n) + [(n - 1, 0)], True)
    lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, 0)
    i = np.arange(n)
    np.testing.assert_array_equal(lv, np.minimum(i, n - i))


def test_closed_form_directed_cycle():
    n = 50
    g = _graph(n, _path(n) + [(n - 1, 0)], False)
    lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, 7)
    np.testing.assert_array_equal(lv, (np.arange(n) - 7) % n)


def test_closed_form_star_and_complete():
    n = 100
    g = _graph(n, [(0, i) for i in range(1, n)], True)
    lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, 5)
    exp = np.full(n, 2)
    exp[5] = 0
    exp[0] = 1
    np.testing.assert_array_equal(lv, exp)
    k = 30
    g = _graph(k, [(i, j) for i in range(k) for j in range(k) if i != j], False)
    lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, 3)
    exp = np.ones(k, dtype=int)
    exp[3] = 0
    np.testing.assert_array_equal(lv, exp)


def test_closed_form_binary_tree():
    n = 1023
    g = _graph(n, [((i - 1) // 2, i) for i in range(1, n)], True)
    lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, 0)
    np.testing.assert_array_equal(lv, np.floor(np.log2(np.arange(n) + 1)).astype(int))


@pytest.mark.parametrize("side", [1, 2, 5, 64])
def test_closed_form_grid_manhattan(side):
    g = gg.lattice(side, p_delete=0.0, shortcut_frac=0.0, seed=1)
    s = (side // 3) * side + side // 2
    lv, par, _ = oracle.bfs(g.row_ptr, g.col_idx, s)
    r, c = np.divmod(np.arange(side * side), side)
    np.testing.assert_array_equal(lv, np.abs(r - s // side) + np.abs(c - s % side))
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, par) is None


@pytest.mark.slow
def test_closed_form_grid_manhattan_4096():
    side = 4096
    g = gg.lattice(side, p_delete=0.0, shortcut_frac=0.0, seed=1)
    assert g.nnz == 2 * 2 * side * (side - 1)
    s = 1234 * side + 3000
    lv, _, nl = oracle.bfs(g.row_ptr, g.col_idx, s)
    r, c = np.divmod(np.arange(side * side, dtype=np.int64), side)
    np.testing.assert_array_equal(lv, np.abs(r - 1234) + np.abs(c - 3000))
    assert nl == (side - 1 - 1234) + 3000 + 1


def test_invariants_rmat14_and_profile():
    g = gg.workload("rmat14").with_csc()
    (s,) = gg.pick_sources(g, 1, 1402)
    lv, par, nl = oracle.bfs(g.row_ptr, g.col_idx, s)
    assert checks.check_levels(g.row_ptr, g.col_idx, s, lv) is None
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, par) is None
    prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, lv)
    reached = (lv >= 0).sum()
    assert prof["nF"].sum() == reached
    assert len(prof["nF"]) == nl
    # |U_k| = n - |P_k| with P_k the union of F_0..F_k
    np.testing.assert_array_equal(prof["nU"], g.n - np.cumsum(prof["nF"]))
    assert (prof["eScan"] <= prof["eU"]).all()
    deg = g.out_degree()
    for k in range(nl):
        F, P = checks.frontiers_from_levels(lv, k)
        assert prof["eF"][k] == deg[F].sum()
        assert prof["eU"][k] == deg[~P].sum()  # symmetric: in-degree = out-degree
        if k:
            _, Pm = checks.frontiers_from_levels(lv, k - 1)
            np.testing.assert_array_equal(F, P & ~Pm)


def test_profile_scan_brute_force():
    # eScan by a direct loop over a small directed graph
    g = gg.directed_random(60, 200, seed=9)
    lv, _, nl = oracle.bfs(g.row_ptr, g.col_idx, 0)
    prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, lv)
    for k in range(nl):
        tot = 0
        for v in range(g.n):
            if 0 <= lv[v] <= k:
                continue
            cnt = 0
            for j in range(g.csc_ptr[v], g.csc_ptr[v + 1]):
                cnt += 1
                if lv[g.csc_idx[j]] == k:
                    break
            tot += cnt
        assert prof["eScan"][k] == tot


def test_profile_hand_worked_example():
    """Per-level counts of a 7-vertex directed graph worked out by hand
    (tests/golden/level_profile_hand_example.json): a wrong scan convention
    (the hit not counted, descending lists, stopping at a visited vertex),
    out- for in-degrees in eU, or U_k taken to include F_k all fail it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "level_profile_hand_example.json")) as f:
        ex = json.load(f)
    g = gg.from_edge_list(ex["n"], ex["edges"], False)
    lv, _, nl = oracle.bfs(g.row_ptr, g.col_idx, ex["source"])
    np.testing.assert_array_equal(lv, ex["depths"])
    prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, lv)
    for key in ("nF", "eF", "nU", "eU", "eScan"):
        np.testing.assert_array_equal(prof[key], ex[key], err_msg=key)


def test_directed_graph_invariants():
    g = gg.directed_random(5000, 20000, seed=3, self_loops=True, duplicates=True)
    for s in (0, 17, 4999):
        lv, par, _ = oracle.bfs(g.row_ptr, g.col_idx, s)
        assert checks.check_levels(g.row_ptr, g.col_idx, s, lv) is None
        assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, par) is None


def test_validators_reject_planted_mistakes():
    g = gg.workload("rmat14")
    (s,) = gg.pick_sources(g, 1, 1402)
    lv, par, _ = oracle.bfs(g.row_ptr, g.col_idx, s)
    reached = np.nonzero((lv > 1))[0]
    v = int(reached[0])
    bad = lv.copy(); bad[v] += 1
    assert checks.check_levels(g.row_ptr, g.col_idx, s, bad) is not None
    bad = lv.copy(); bad[v] -= 1
    assert checks.check_levels(g.row_ptr, g.col_idx, s, bad) is not None
    bad = lv.copy(); bad[v] = -1
    assert checks.check_levels(g.row_ptr, g.col_idx, s, bad) is not None
    p = par.copy(); p[s] = int(par[v])
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, p) is not None
    # a parent one level up but not adjacent
    same = np.nonzero(lv == lv[v] - 1)[0]
    nbrs = set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist())
    nonadj = [int(u) for u in same if int(u) not in nbrs]
    p = par.copy(); p[v] = nonadj[0]
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, p) == "parent edge not in the graph"
    p = par.copy(); p[v] = v
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, p) is not None
    unreached = np.nonzero(lv < 0)[0]
    p = par.copy(); p[int(unreached[0])] = s
    assert checks.check_parents(g.row_ptr, g.col_idx, s, lv, p) is not None


def test_planted_oracle_bug_is_caught_by_brute_force():
    """A plausible oracle mistake (assigning depth at dequeue instead of at
    discovery, which lets a vertex be enqueued twice with a larger depth)
    disagrees with brute force on a small graph."""
    def buggy(n, edges, s):
        adj = [[] for _ in range(n)]
        for a, b in edges:
            adj[a].append(b)
        lv = [-1] * n
        q = [(s, 0)]
        while q:
            u, d = q.pop()  # LIFO: depth-first order, a plausible slip
            if lv[u] != -1:
                continue
            lv[u] = d
            for w in adj[u]:
                if lv[w] == -1:
                    q.append((w, d + 1))
        return np.array(lv)
    edges = [(0, 1), (1, 2), (2, 3), (0, 3), (1, 0), (2, 1), (3, 2), (3, 0)]
    ref = brute.levels_from(4, edges, 0)
    assert not np.array_equal(buggy(4, edges, 0), ref)


def test_multi_and_batch_loops():
    g = gg.workload("rmat14")
    srcs = gg.pick_sources(g, 5, 77)
    M = oracle.multi(g.row_ptr, g.col_idx, srcs)
    for i, s in enumerate(srcs):
        np.testing.assert_array_equal(M[i], oracle.bfs(g.row_ptr, g.col_idx, s)[0])
    b = gg.concat([gg.rmat(8, seed=3), gg.lattice(9, seed=4)], [1, 2])
    out = oracle.batch(b.graphs, b.sources)
    assert out.shape[0] == b.total_n
    np.testing.assert_array_equal(out[: b.graphs[0].n],
                                  oracle.bfs(b.graphs[0].row_ptr, b.graphs[0].col_idx, 1)[0])
