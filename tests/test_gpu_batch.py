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


CONFIGS = [B.api.BatchConfig(256, 0, 256, 1), B.api.BatchConfig(256, 4096, 512, 2),
           B.api.BatchConfig(512, 65536, 512, 2), B.api.BatchConfig(1024, 131072, 2048, 1),
           B.api.BatchConfig(1024, 0, 1024, 2)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"t{c.block_threads}_s{c.small_vertices}_c{c.chunk_vertices}")
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
    for cfg in (B.api.BatchConfig(256, 0, 256, 1), B.api.BatchConfig(1024, 0, 2048, 2)):
        lv, _ = B.bfs_batch(B.DeviceBatch(b), config=cfg)
        _check(b, lv)


def test_batch_directed_instances_push_only():
    graphs = [gg.directed_random(500 + 50 * i, 3000, seed=i, self_loops=True, duplicates=True) for i in range(8)]
    b = gg.concat(graphs, [i for i in range(8)])
    lv, _ = B.bfs_batch(B.DeviceBatch(b))
    _check(b, lv)


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
        B.bfs_batch(db, config=B.api.BatchConfig(300, 0, 300, 1))
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
