"""bfs_levels_noalloc (the allocation-free variant of bfs_levels, scratch in
a static device array) against bfs_levels through the C ABI: identical
depths and counts on two calls in a row, the second on a smaller graph, for
the automatic and fixed modes, a schedule and a renumbered graph; and the
oracle agrees."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402
from paper_2607_17106_amd import selector  # noqa: E402


def _pair(g, s, **kw):
    dg = B.DeviceGraph.from_graph(g)
    ref, st_ref = B.bfs_levels(dg, int(s), **kw)
    got, st = B.bfs_levels_noalloc(dg, int(s), **kw)
    return dg, ref.cpu().numpy(), st_ref, got.cpu().numpy(), st


@pytest.mark.parametrize("mode", [B.AUTO_HEURISTIC, B.AUTO_LEARNED, B.PUSH_Q_MERGE, B.PULL_B, B.PUSH_B_NOATOMIC,
                                  "schedule"])
def test_noalloc_matches_bfs_levels_twice(mode):
    loaded = selector.load_default() if mode == B.AUTO_LEARNED else False
    try:
        kw = dict(variant=mode)
        if mode == "schedule":
            kw = dict(variant=B.SCHEDULE, schedule=[B.PUSH_Q_BLOCK, B.PUSH_B_ATOMIC, B.PULL_B, B.PUSH_Q_THREAD])
        # the larger graph first, then a smaller one: the scratch keeps the
        # first call's contents
        for g in (gg.rmat(18, seed=1811), gg.lattice(40, seed=12)):
            s = int(gg.pick_sources(g, 1, 7)[0])
            _, ref, st_ref, got, st = _pair(g, s, **kw)
            np.testing.assert_array_equal(got, ref, err_msg=f"{g.name} mode={mode}")
            np.testing.assert_array_equal(got, oracle.bfs(g.row_ptr, g.col_idx, s, want_parents=False)[0])
            for key in ("num_levels", "reached", "component_edges"):
                assert st[key] == st_ref[key], key
    finally:
        if loaded:
            B.selector_clear()


def test_noalloc_renumbered_graph_and_directed():
    g = gg.rmat(16, seed=1611)
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, _ = B.reorder_degree(dg)
    s = int(gg.pick_sources(g, 1, 9)[0])
    ref, _ = B.bfs_levels(rg, s, vertex_map=new_of_old)
    got, _ = B.bfs_levels_noalloc(rg, s, vertex_map=new_of_old)
    np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
    d = gg.directed_random(3000, 12000, seed=5, self_loops=True, duplicates=True)
    dd = B.DeviceGraph.from_graph(d)
    for s in (0, 1234):
        ref, _ = B.bfs_levels(dd, s)
        got, _ = B.bfs_levels_noalloc(dd, s)
        np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_rejections():
    g = gg.rmat(10, seed=3)
    dg = B.DeviceGraph.from_graph(g)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels_noalloc(dg, 0, flags=B.F_LEVEL_STATS)
    assert e.value.code == -7
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels_noalloc(dg, g.n)
    assert e.value.code == -1
