"""The tunable choices of the 64-lane multi-source search (bfs_multi_config)
and its autotuner: every configuration returns the oracle's depths row for
row (the choices change the launch shapes, tile cuts, round caps, direction
and split switches, never the result), the autotuner returns values from its
candidate sets and stores them for the graph, and the next call with no
configuration, which uses the stored one, is exact too."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402

CONFIGS = [
    B.MultiConfig(),                              # the defaults
    B.MultiConfig(wide_ratio=1),                  # one vertex per thread on every non-split bottom-up level
    B.MultiConfig(wide_ratio=1 << 20),            # four per thread on every one
    B.MultiConfig(split_vpt=1),
    B.MultiConfig(cap0=1),                        # smallest first round: many rounds
    B.MultiConfig(cap0=1 << 20),                  # one round
    B.MultiConfig(tile_alpha=16),                 # smallest tiles
    B.MultiConfig(tile_alpha=1024),               # largest tiles (VPT=4 groups span 4096 light vertices' weight)
    B.MultiConfig(alpha=1),                       # bottom-up almost never
    B.MultiConfig(alpha=1000),                    # bottom-up as soon as the frontier holds n/8 out-edges
    B.MultiConfig(split_lout=1, wide_ratio=2),
    B.MultiConfig(split_lout=1 << 20, split_vpt=1, cap0=7, tile_alpha=17),
    B.MultiConfig(wide_vpt=2, narrow_vpt=2, split_vpt=2),
    B.MultiConfig(wide_ratio=1, wide_vpt=4, narrow_vpt=1),
    B.MultiConfig(wide_ratio=1 << 20, narrow_vpt=1, split_vpt=2, cap0=3),
]


def _graphs():
    yield "rmat14", gg.workload("rmat14"), None
    yield "lattice", gg.lattice(120, seed=3), None
    yield "directed", gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True), \
        np.arange(0, 3000, 47)[:64]
    rng = np.random.default_rng(11)
    n = 9000
    src = np.concatenate([rng.integers(0, n, 30000), np.full(3000, 7), rng.integers(0, n, 2600)])
    dst = np.concatenate([rng.integers(0, n, 30000), rng.integers(0, n, 3000), np.full(2600, 4242)])
    yield "directed_hubs", gg.from_edge_list(n, np.stack([src, dst], 1), False), np.array([7, 4242, 1, 2, 3, 100])


def test_every_config_gives_the_oracle_depths():
    for name, g, srcs in _graphs():
        if srcs is None:
            srcs = gg.pick_sources(g, 64, 5)
        ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
        dg = B.DeviceGraph.from_graph(g)
        for cfg in CONFIGS:
            lv, _ = B.bfs_multi(dg, srcs, config=cfg)
            np.testing.assert_array_equal(lv.cpu().numpy(), ref, err_msg=f"{name} {cfg}")


def test_every_config_on_the_degree_ordered_graph():
    """The renumbered graph (split levels on, vertex_map for the columns),
    a ragged group of 70 sources (a full group and one of 6)."""
    g = gg.workload("rmat14")
    srcs = gg.pick_sources(g, 70, 9)
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, _ = B.reorder_degree(dg)
    for cfg in CONFIGS:
        lv, _ = B.bfs_multi(rg, srcs, vertex_map=new_of_old, config=cfg)
        np.testing.assert_array_equal(lv.cpu().numpy(), ref, err_msg=str(cfg))


def test_autotune_stores_a_config_the_next_call_uses():
    g = gg.workload("rmat14")
    srcs = gg.pick_sources(g, 64, 5)
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    dg = B.DeviceGraph.from_graph(g)
    rg, new_of_old, _ = B.reorder_degree(dg)
    cfg, ms = B.bfs_multi_autotune(rg, srcs, vertex_map=new_of_old)
    assert ms > 0
    assert cfg.wide_ratio in (2, 4, 8, 16, 64, 1 << 20)
    assert cfg.split_vpt in (1, 2, 4) and cfg.wide_vpt in (1, 2, 4) and cfg.narrow_vpt in (1, 2, 4)
    assert cfg.cap0 in (16, 32, 64, 128)
    assert cfg.tile_alpha in (32, 64, 128)
    assert cfg.alpha in (4, 7, 14)
    assert cfg.split_lout in (4, 16, 64)
    lv, _ = B.bfs_multi(rg, srcs, vertex_map=new_of_old)  # the stored configuration
    np.testing.assert_array_equal(lv.cpu().numpy(), ref)
    lv, _ = B.bfs_multi(rg, srcs, vertex_map=new_of_old, config=cfg)
    np.testing.assert_array_equal(lv.cpu().numpy(), ref)


def test_config_errors():
    g = gg.rmat(10, seed=3)
    dg = B.DeviceGraph.from_graph(g)
    for bad in (B.MultiConfig(split_vpt=3), B.MultiConfig(wide_vpt=8), B.MultiConfig(narrow_vpt=-1),
                B.MultiConfig(tile_alpha=8), B.MultiConfig(tile_alpha=2048),
                B.MultiConfig(cap0=-1), B.MultiConfig(wide_ratio=-3), B.MultiConfig(alpha=-1),
                B.MultiConfig(split_lout=-2)):
        with pytest.raises(B.BfsError) as e:
            B.bfs_multi(dg, np.array([0, 1]), config=bad)
        assert e.value.code == -1, bad
