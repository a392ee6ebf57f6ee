"""GPU parity of the batched persistent BFS: every instance's depths equal the
oracle BFS on that instance alone, for several launch configurations and
after autotuning; edges never cross instances."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402


def _small_batch(seed=3):
    graphs, srcs = [], []
    rng = np.random.default_rng(seed)
    for i in range(48):
        kind = i % 4
        if kind == 0:
            g = gg.rmat(int(rng.integers(6, 13)), seed=100 + i)
        elif kind == 1:
            g = gg.lattice(int(rng.integers(8, 90)), seed=200 + i)
        elif kind == 2:
            g = gg.erdos_renyi(int(rng.integers(50, 3000)), 4.0, seed=300 + i)
        else:
            g = gg.from_edge_list(int(rng.integers(6, 40)), [(j, j + 1) for j in range(int(rng.integers(0, 5)))], True)
        s = gg.pick_sources(g, 1, i)
        graphs.append(g)
        srcs.append(int(s[0]) if len(s) else 0)
    # a hub-heavy instance and a single vertex
    graphs.append(gg.from_edge_list(6000, [(0, j) for j in range(1, 6000)] + [(5, 6), (6, 7)], True))
    srcs.append(7)
    graphs.append(gg.from_edge_list(1, [], True))
    srcs.append(0)
    return gg.concat(graphs, srcs)


def _check(b, lv):
    lv = lv.cpu().numpy()
    ref = oracle.batch(b.graphs, b.sources)
    for i in range(b.num):
        a, z = int(b.v_off[i]), int(b.v_off[i + 1])
        np.testing.assert_array_equal(lv[a:z], ref[a:z], err_msg=f"instance {i}")
    return ref


# (threads, small_vertices, blocks/CU, team_vertices, max_team): single
# workgroups with the visited bitmap in LDS, one-member teams, and teams of up
# to 16 workgroups
CONFIGS = [B.api.BatchConfig(256, 0, 1, 0, 1), B.api.BatchConfig(256, 4096, 2, 1024, 4),
           B.api.BatchConfig(512, 65536, 2), B.api.BatchConfig(1024, 1 << 20, 1),
           B.api.BatchConfig(1024, 0, 2, 512, 16), B.api.BatchConfig(512, 64, 4, 256, 8)]


def _cid(c):
    return f"t{c.block_threads}_s{c.small_vertices}_tv{c.team_vertices}_g{c.max_team}"


@pytest.mark.parametrize("cfg", CONFIGS, ids=_cid)
def test_batch_matches_oracle(cfg):
    b = _small_batch()
    db = B.DeviceBatch(b)
    lv, st = B.bfs_batch(db, config=cfg)
    ref = _check(b, lv)
    comp = sum(oracle.edges_in_component(g.row_ptr, ref[int(b.v_off[i]):int(b.v_off[i + 1])])
               for i, g in enumerate(b.graphs))
    assert st["component_edges"] == comp


def test_batch_odd_largest_instance_global_bitmaps():
    """The largest instance has an odd vertex count (a 91 x 91 lattice, 8281
    vertices) and every instance keeps its bitmaps in global scratch
    (small_vertices 0): the bitmaps' 64-bit atomics must stay aligned."""
    graphs = [gg.lattice(91, seed=17), gg.rmat(9, seed=5), gg.lattice(33, seed=2), gg.from_edge_list(3, [(0, 1)], True)]
    srcs = [int(gg.pick_sources(g, 1, 3)[0]) if g.n > 3 else 0 for g in graphs]
    b = gg.concat(graphs, srcs)
    assert max(g.n for g in graphs) % 2 == 1
    for cfg in (B.api.BatchConfig(256, 0, 1, 0, 1), B.api.BatchConfig(1024, 0, 2, 0, 1), B.api.BatchConfig(1024, 8192, 2)):
        lv, _ = B.bfs_batch(B.DeviceBatch(b), config=cfg)
        _check(b, lv)


def test_batch_directed_instances_push_only():
    graphs = [gg.directed_random(500 + 50 * i, 3000, seed=i, self_loops=True, duplicates=True) for i in range(8)]
    b = gg.concat(graphs, [i for i in range(8)])
    db = B.DeviceBatch(b)
    lv, _ = B.bfs_batch(db)
    _check(b, lv)
    for cfg in (B.api.BatchConfig(256, 0, 1, 128, 6), B.api.BatchConfig(1024, 0, 2, 0, 1), B.api.BatchConfig(1024, 1 << 20, 1)):
        lv, _ = B.bfs_batch(db, config=cfg)
        _check(b, lv)


@pytest.mark.parametrize("cfg", [B.api.BatchConfig(256, 0, 2, 2048, 16), B.api.BatchConfig(1024, 0, 1, 0, 1),
                                 B.api.BatchConfig(512, 1000, 2, 4096, 3), B.api.BatchConfig(1024, 1 << 20, 2)],
                         ids=_cid)
def test_batch_team_giant_vertices(cfg):
    """Vertices of out-degree above the team kernel's giant threshold (8192):
    listed when found and expanded by every member in slices -- a hub found at
    level 1, a hub that is the source, two hubs joined by a path, and a
    directed hub with in-degree but no out-edges."""
    graphs, srcs = [], []
    graphs.append(gg.from_edge_list(20000, [(0, j) for j in range(1, 20000)] + [(7, 8)], True))
    srcs.append(5)
    graphs.append(gg.from_edge_list(20000, [(0, j) for j in range(1, 20000)], True))
    srcs.append(0)
    e = [(0, j) for j in range(1, 9500)] + [(9500, j) for j in range(9501, 19000)] + [(1, 2), (2, 9501)]
    graphs.append(gg.from_edge_list(19100, e, True))
    srcs.append(19000 - 1)
    graphs.append(gg.lattice(70, seed=9))
    srcs.append(0)
    b = gg.concat(graphs, srcs)
    lv, st = B.bfs_batch(B.DeviceBatch(b), config=cfg)
    ref = _check(b, lv)
    comp = sum(oracle.edges_in_component(g.row_ptr, ref[int(b.v_off[i]):int(b.v_off[i + 1])])
               for i, g in enumerate(b.graphs))
    assert st["component_edges"] == comp


def test_batch_workspace_size_and_caller_workspace():
    b = _small_batch(seed=8)
    db = B.DeviceBatch(b)
    cfg = B.api.BatchConfig(512, 1024, 2, 2048, 4)
    need = B.api.batch_workspace_size(db, cfg)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    lv, _ = B.bfs_batch(db, config=cfg, workspace=ws)
    _check(b, lv)
    with pytest.raises(B.BfsError) as e:
        B.bfs_batch(db, config=cfg, workspace=ws[:need - 1])
    assert e.value.code == -3


def test_batch_autotune_then_run():
    b = _small_batch(seed=5)
    db = B.DeviceBatch(b)
    cfg, ms = B.bfs_batch_autotune(db)
    assert ms > 0 and cfg.block_threads in (256, 512, 1024)
    lv, _ = B.bfs_batch(db)  # uses the cached tuned config
    _check(b, lv)


def test_batch_errors():
    b = _small_batch()
    db = B.DeviceBatch(b)
    bad = b.sources.copy()
    bad[3] = b.graphs[3].n
    with pytest.raises(B.BfsError) as e:
        B.bfs_batch(db, sources=bad)
    assert e.value.code == -1
    with pytest.raises(B.BfsError) as e:
        B.bfs_batch(db, config=B.api.BatchConfig(300, 0, 1))
    assert e.value.code == -1


@pytest.mark.slow
def test_mixed_batch_512_every_instance():
    """The benchmark's 512-instance mix (R-MAT 10-18, lattices 128^2-1024^2):
    every instance equal to the oracle on that instance alone."""
    b = gg.mixed_batch(512, seed=5501)
    db = B.DeviceBatch(b)
    lv, st = B.bfs_batch(db)
    got = lv.cpu().numpy()
    ref = oracle.batch(b.graphs, b.sources)
    for i in range(b.num):
        a, z = int(b.v_off[i]), int(b.v_off[i + 1])
        np.testing.assert_array_equal(got[a:z], ref[a:z], err_msg=f"instance {i}")
    comp = sum(oracle.edges_in_component(g.row_ptr, ref[int(b.v_off[i]):int(b.v_off[i + 1])])
               for i, g in enumerate(b.graphs))
    assert st["component_edges"] == comp
