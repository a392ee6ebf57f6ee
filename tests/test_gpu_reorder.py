"""GPU parity of the renumberings (bfs_reorder_degree, bfs_reorder_rcm) and of
the multi-source search run on a renumbered graph through options.vertex_map.

* the maps and the renumbered CSR / CSC equal the oracle's (oracle/reorder.py)
  element by element: the order and the sorted rows are unique;
* bfs_multi on the renumbered graph with vertex_map returns, row for row, the
  oracle's depths on the ORIGINAL graph from the original sources;
* the launch the benchmark times (R-MAT scale 22, 64 sources, renumbered)
  against the oracle on sampled rows;
* errors: vertex_map on the other entry points, malformed graphs.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import reorder as ro

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402

MODES = [B.AUTO_HEURISTIC, B.PUSH_Q_BLOCK, B.PULL_B]


def _graphs():
    yield "rmat12", gg.rmat(12, seed=77)
    yield "directed", gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True)
    yield "lattice", gg.lattice(90, seed=3)
    yield "isolated", gg.from_edge_list(5, [(1, 2)], True)
    yield "one_vertex", gg.from_edge_list(1, [], True)
    yield "ragged", gg.rmat(9, seed=2)  # 512 vertices, many of degree 0
    yield "path701", gg.from_edge_list(701, [(i, i + 1) for i in range(700)], True)


@pytest.mark.parametrize("name,g", list(_graphs()))
def test_reorder_matches_oracle(name, g):
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, old_of_new = B.reorder_degree(dg)
    n2o, o2n = ro.degree_order(g.row_ptr)
    np.testing.assert_array_equal(new_of_old.cpu().numpy(), n2o, err_msg=name)
    np.testing.assert_array_equal(old_of_new.cpu().numpy(), o2n, err_msg=name)
    rp, ci = ro.renumber(g.row_ptr, g.col_idx, n2o)
    np.testing.assert_array_equal(rg.row_ptr.cpu().numpy(), rp, err_msg=name)
    np.testing.assert_array_equal(rg.col_idx.cpu().numpy(), ci, err_msg=name)
    if not g.symmetric:
        g.with_csc()
        cp, cx = ro.renumber(g.csc_ptr, g.csc_idx, n2o)
        np.testing.assert_array_equal(rg.csc_ptr.cpu().numpy(), cp, err_msg=name)
        np.testing.assert_array_equal(rg.csc_idx.cpu().numpy(), cx, err_msg=name)
    else:
        assert rg.csc_ptr.data_ptr() == rg.row_ptr.data_ptr()


def _check_mapped(g, srcs, variant, hub_split=0):
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, _ = B.reorder_degree(dg)
    lv, st = B.bfs_multi(rg, srcs, variant=variant, vertex_map=new_of_old, hub_split=hub_split)
    lv = lv.cpu().numpy()
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    for i in range(len(srcs)):
        np.testing.assert_array_equal(lv[i], ref[i], err_msg=f"lane {i} source {srcs[i]} mode {variant}")
    assert st["reached"] == int((ref >= 0).sum())
    assert st["component_edges"] == sum(oracle.edges_in_component(g.row_ptr, ref[i]) for i in range(len(srcs)))


@pytest.mark.parametrize("variant", MODES)
def test_mapped_multi_matches_oracle(variant):
    g = gg.workload("rmat14")
    _check_mapped(g, gg.pick_sources(g, 64, 5), variant)
    g = gg.rmat(12, seed=77)
    srcs = gg.pick_sources(g, 50, 6)
    _check_mapped(g, np.concatenate([srcs, srcs[:20]]), variant)  # two groups, duplicates
    _check_mapped(g, srcs[:1], variant)
    g = gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True)
    _check_mapped(g, np.arange(0, 3000, 47)[:64], variant)
    g = gg.from_edge_list(5, [(1, 2)], True)
    _check_mapped(g, np.array([0, 1, 4]), variant)


@pytest.mark.parametrize("variant", [B.AUTO_HEURISTIC, B.PULL_B])
def test_mapped_split_levels(variant):
    """Renumbered graphs with vertex_map and split bottom-up levels at ids
    around the hub block (every bottom-up level split)."""
    g = gg.workload("rmat14")
    srcs = gg.pick_sources(g, 64, 5)
    for t in (1, 16, 100, 1000, 5000):
        _check_mapped(g, srcs, variant, hub_split=t)
    g = gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True)
    _check_mapped(g, np.arange(0, 3000, 47)[:64], variant, hub_split=40)


@pytest.mark.parametrize("variant", MODES)
def test_mapped_long_paths(variant):
    """Depths above 255 (flush passes, whose bookkeeping is per output column)."""
    for n in (700, 701):
        g = gg.from_edge_list(n, [(i, i + 1) for i in range(n - 1)], True)
        _check_mapped(g, np.array([0, n - 1, 350, 100, 0, 3]), variant)


@pytest.mark.parametrize("variant", [B.AUTO_HEURISTIC, B.PUSH_Q_BLOCK, B.PULL_B, B.PUSH_B_NOATOMIC])
def test_single_source_vertex_map(variant):
    """bfs_levels / bfs_parents on the renumbered graph with vertex_map: the
    oracle's depths on the original graph from the original source, and
    parents (original ids) that pass the validity checks there."""
    from oracle import checks
    graphs = [gg.workload("rmat14"), gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True),
              gg.from_edge_list(701, [(i, i + 1) for i in range(700)], True), gg.from_edge_list(5, [(1, 2)], True)]
    for g in graphs:
        dg = B.DeviceGraph.from_graph(g)
        for reorder in (B.reorder_degree, B.reorder_rcm):
            rg, new_of_old, _ = reorder(dg)
            for s in (0, g.n - 1, g.n // 2):
                ref = oracle.bfs(g.row_ptr, g.col_idx, s, want_parents=False)[0]
                lv, _ = B.bfs_levels(rg, s, variant=variant, vertex_map=new_of_old)
                np.testing.assert_array_equal(lv.cpu().numpy(), ref, err_msg=f"{reorder.__name__} source {s}")
                lv, par, _ = B.bfs_parents(rg, s, variant=variant, vertex_map=new_of_old)
                np.testing.assert_array_equal(lv.cpu().numpy(), ref)
                assert checks.check_parents(g.row_ptr, g.col_idx, s, ref, par.cpu().numpy()) is None


def test_vertex_map_rejected_by_step_time():
    g = gg.rmat(10, seed=3)
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, _ = B.reorder_degree(dg)
    depths = torch.from_numpy(oracle.bfs(rg.row_ptr.cpu().numpy(), rg.col_idx.cpu().numpy(), 0,
                                         want_parents=False)[0]).cuda()
    lib = B.load()
    opt = B._lib.BfsOptions()
    opt.vertex_map = new_of_old.data_ptr()
    import ctypes
    ms = ctypes.c_float(0)
    scratch = torch.empty(g.n, dtype=torch.int32, device="cuda")
    rc = lib.bfs_step_time(rg.c, ctypes.c_void_p(depths.data_ptr()), 0, B.PUSH_Q_BLOCK, 1,
                           ctypes.c_void_p(scratch.data_ptr()), ctypes.byref(opt), ctypes.byref(ms),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -7


def test_reorder_rejects_malformed_graph():
    g = gg.rmat(8, seed=1)
    bad = g.col_idx.copy()
    bad[3] = g.n + 5
    dg = B.DeviceGraph(g.n, g.row_ptr, bad, symmetric=True)
    with pytest.raises(B.BfsError) as e:
        B.reorder_degree(dg)
    assert e.value.code == -2


_RMAT22 = {}


def _rmat22_reference():
    """R-MAT scale 22, its 64 sources and every oracle row (one search per
    host thread), computed once for the tests below."""
    if not _RMAT22:
        g = gg.workload("rmat22")
        nsrc, sseed = gg.WORKLOAD_SOURCES["rmat22"]
        srcs = gg.pick_sources(g, nsrc, sseed)
        _RMAT22.update(g=g, srcs=srcs, ref=oracle.multi(g.row_ptr, g.col_idx, srcs))
    return _RMAT22["g"], _RMAT22["srcs"], _RMAT22["ref"]


def test_rmat22_64_sources_every_row():
    """The benchmark's launch: R-MAT scale 22, its 64 sources, the renumbered
    graph with vertex_map, default heuristic: every row equal to the oracle on
    the original graph.  Then the same search on the graph as generated."""
    g, srcs, ref = _rmat22_reference()
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, _ = B.reorder_degree(dg)
    lv, st = B.bfs_multi(rg, srcs, vertex_map=new_of_old, level_stats=True)
    # the sparse hub frontier after the first level takes a split level
    assert np.any(st["variant"][:st["num_levels"]] == B.MS_SPLIT)
    got = lv.cpu().numpy()
    del lv, rg, new_of_old
    for i in range(len(srcs)):
        np.testing.assert_array_equal(got[i], ref[i], err_msg=f"renumbered row {i}")
    lv, _ = B.bfs_multi(dg, srcs)
    got = lv.cpu().numpy()
    del lv
    for i in range(len(srcs)):
        np.testing.assert_array_equal(got[i], ref[i], err_msg=f"input-order row {i}")


# ------------------------------------------------------------- RCM
@pytest.mark.parametrize("name,g", list(_graphs()))
def test_rcm_matches_oracle(name, g):
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, old_of_new = B.reorder_rcm(dg)
    if g.symmetric:
        n2o, o2n = ro.rcm_order(g.row_ptr, g.col_idx)
    else:
        g.with_csc()
        n2o, o2n = ro.rcm_order(g.row_ptr, g.col_idx, g.csc_ptr, g.csc_idx)
    np.testing.assert_array_equal(old_of_new.cpu().numpy(), o2n, err_msg=name)
    np.testing.assert_array_equal(new_of_old.cpu().numpy(), n2o, err_msg=name)
    rp, ci = ro.renumber(g.row_ptr, g.col_idx, n2o)
    np.testing.assert_array_equal(rg.row_ptr.cpu().numpy(), rp, err_msg=name)
    np.testing.assert_array_equal(rg.col_idx.cpu().numpy(), ci, err_msg=name)
    if not g.symmetric:
        cp, cx = ro.renumber(g.csc_ptr, g.csc_idx, n2o)
        np.testing.assert_array_equal(rg.csc_ptr.cpu().numpy(), cp, err_msg=name)
        np.testing.assert_array_equal(rg.csc_idx.cpu().numpy(), cx, err_msg=name)
    assert not getattr(rg, "hub_order", False)


@pytest.mark.parametrize("variant", MODES)
def test_rcm_mapped_multi_matches_oracle(variant):
    for g, srcs in ((gg.rmat(12, seed=77), None), (gg.directed_random(3000, 15000, seed=4), np.arange(0, 3000, 47)[:64]),
                    (gg.lattice(90, seed=3), None)):
        if srcs is None:
            srcs = gg.pick_sources(g, 64, 6)
        dg = B.DeviceGraph.from_graph(g)
        rg, new_of_old, _ = B.reorder_rcm(dg)
        lv, st = B.bfs_multi(rg, srcs, variant=variant, vertex_map=new_of_old)
        ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
        np.testing.assert_array_equal(lv.cpu().numpy(), ref)


def test_rcm_rmat22_every_row():
    """R-MAT scale 22 renumbered by RCM, its 64 sources through vertex_map:
    every row equal to the oracle on the original graph."""
    g, srcs, ref = _rmat22_reference()
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, old_of_new = B.reorder_rcm(dg)
    del dg
    o2n = old_of_new.cpu().numpy()
    assert np.array_equal(np.sort(o2n), np.arange(g.n))
    lv, st = B.bfs_multi(rg, srcs, vertex_map=new_of_old)
    got = lv.cpu().numpy()
    for i in range(len(srcs)):
        np.testing.assert_array_equal(got[i], ref[i], err_msg=f"row {i}")
