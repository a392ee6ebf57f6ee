"""GPU parity of the 64-lane bit-packed multi-source BFS: row i of the output
equals the oracle BFS from source i, bit for bit."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402

MODES = [B.AUTO_HEURISTIC, B.PUSH_Q_BLOCK, B.PULL_B]


def _check(g, srcs, variant, level_stats=False):
    dg = B.DeviceGraph.from_graph(g)
    lv, st = B.bfs_multi(dg, srcs, variant=variant, level_stats=level_stats)
    lv = lv.cpu().numpy()
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    for i in range(len(srcs)):
        np.testing.assert_array_equal(lv[i], ref[i], err_msg=f"lane {i} source {srcs[i]} mode {variant}")
    assert st["component_edges"] == sum(oracle.edges_in_component(g.row_ptr, ref[i]) for i in range(len(srcs)))
    assert st["reached"] == int((ref >= 0).sum())
    if level_stats:
        _check_level_stats(g, np.asarray(srcs), ref, st)
    else:
        assert st["num_levels"] == int(ref.max()) + 1
    return st


def _check_level_stats(g, srcs, ref, st):
    """Per-level entries, group by group, against counts from the oracle's
    depths: lane pairs and vertices found at each level, frontier sizes."""
    i = 0
    for g0 in range(0, len(srcs), 64):
        r = ref[g0:g0 + 64]
        depth_max = int(r.max())
        for k in range(depth_max + 1):
            found = r == k + 1
            assert int(st["next"][i]) == int(found.sum()), (g0, k)
            assert int(st["frontier_ld"][i]) == int(found.any(axis=0).sum()), (g0, k)
            assert int(st["frontier"][i]) == int((r == k).any(axis=0).sum()), (g0, k)
            assert 0 <= int(st["frontier_ld2"][i]) <= int(st["scanned"][i])
            assert 0 <= int(st["scanned_aux"][i]) <= int(st["scanned"][i])
            assert 0 <= int(st["hits_aux"][i]) <= min(int(st["frontier_ld2"][i]), int(st["scanned_aux"][i]))
            i += 1
    assert st["num_levels"] == i


@pytest.mark.parametrize("variant", MODES)
def test_rmat14_64_sources(variant):
    g = gg.workload("rmat14")
    _check(g, gg.pick_sources(g, 64, 5), variant)


@pytest.mark.parametrize("variant", MODES)
def test_ragged_group_sizes_and_duplicates(variant):
    g = gg.rmat(12, seed=77)
    srcs = gg.pick_sources(g, 50, 6)
    srcs70 = np.concatenate([srcs, srcs[:20]])  # 70 sources: one full group of 64 + 6, with duplicates
    _check(g, srcs70, variant)
    _check(g, srcs[:1], variant)
    _check(g, np.array([srcs[0]] * 3), variant)


@pytest.mark.parametrize("variant", MODES)
def test_directed_and_lattice(variant):
    g = gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True)
    _check(g, np.arange(0, 3000, 47)[:64], variant)
    g = gg.lattice(120, seed=3)
    _check(g, gg.pick_sources(g, 33, 8), variant)
    g = gg.from_edge_list(5, [(1, 2)], True)  # isolated sources
    _check(g, np.array([0, 1, 4]), variant)


@pytest.mark.parametrize("variant", MODES)
def test_long_paths_cross_depth_windows(variant):
    """Depths above 255 take more than one window of depth planes (flush
    passes between windows)."""
    for n in (700, 701):  # 16-byte row stores, and the unaligned fallback
        g = gg.from_edge_list(n, [(i, i + 1) for i in range(n - 1)], True)
        _check(g, np.array([0, n - 1, 350, 100, 0, 3]), variant, level_stats=True)
    g = gg.lattice(200, p_delete=0.0, shortcut_frac=0.0, seed=1)
    _check(g, np.array([0, 199, 200 * 200 - 1, 20100]), variant)


@pytest.mark.parametrize("variant", MODES)
def test_directed_hubs(variant):
    """Directed graph whose heavy in-degree and heavy out-degree vertices
    differ (separate chunk lists for the two directions)."""
    rng = np.random.default_rng(11)
    n = 9000
    e = [rng.integers(0, n, 30000), rng.integers(0, n, 30000)]
    src = np.concatenate([e[0], np.full(3000, 7), rng.integers(0, n, 2600)])
    dst = np.concatenate([e[1], rng.integers(0, n, 3000), np.full(2600, 4242)])
    g = gg.from_edge_list(n, np.stack([src, dst], 1), False)
    deg_out = np.diff(g.row_ptr)
    deg_in = np.diff(g.csc_ptr)
    assert deg_out[7] > 2048 and deg_in[4242] > 2048 and deg_in[7] < 2048 and deg_out[4242] < 2048
    _check(g, np.array([7, 4242, 1, 2, 3, 100, 7]), variant, level_stats=True)


@pytest.mark.parametrize("variant", MODES)
def test_level_stats(variant):
    g = gg.rmat(12, seed=77)
    srcs = gg.pick_sources(g, 50, 6)
    _check(g, np.concatenate([srcs, srcs[:20]]), variant, level_stats=True)


@pytest.mark.parametrize("variant", [B.AUTO_HEURISTIC, B.PULL_B])
def test_large_sparse_graph(variant):
    """n above 2^23: the frontier summary groups span more than one bitmap
    word; most vertices isolated (depth -1 in every row)."""
    rng = np.random.default_rng(12)
    n = 9_000_000
    a = rng.integers(0, 2_000_000, 400_000)
    b = rng.integers(0, 2_000_000, 400_000)
    c = rng.integers(0, n, 100_000)
    d = rng.integers(0, n, 100_000)
    g = gg.from_edge_list(n, np.stack([np.concatenate([a, c]), np.concatenate([b, d])], 1), True)
    _check(g, gg.pick_sources(g, 8, 13), variant, level_stats=True)


def test_multi_errors():
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    with pytest.raises(B.BfsError) as e:
        B.bfs_multi(dg, np.array([], dtype=np.int32))
    assert e.value.code == -1
    with pytest.raises(B.BfsError) as e:
        B.bfs_multi(dg, np.array([0, g.n]))
    assert e.value.code == -1
    dnc = B.DeviceGraph(g.n, g.row_ptr, g.col_idx)
    with pytest.raises(B.BfsError) as e:
        B.bfs_multi(dnc, np.array([0]))
    assert e.value.code == -7


def test_rmat20_sampled_rows():
    """Full-size-style check: 64 sources on a scale-20 graph, every row against
    the oracle (each oracle BFS takes ~0.1 s)."""
    g = gg.rmat(20, seed=4020)
    srcs = gg.pick_sources(g, 64, 9)
    dg = B.DeviceGraph.from_graph(g)
    lv, st = B.bfs_multi(dg, srcs)
    lv = lv.cpu().numpy()
    for i in range(0, 64, 7):
        np.testing.assert_array_equal(lv[i], oracle.bfs(g.row_ptr, g.col_idx, int(srcs[i]))[0])


def test_level_timing_fills_ms():
    """With per-level timing every level of every group gets its step time and
    its main kernel's time (read back after the next level is enqueued), within
    the call's own time; more than 16 levels reuse the event ring."""
    for g, srcs in ((gg.workload("rmat14"), None), (gg.from_edge_list(300, [(i, i + 1) for i in range(299)], True),
                                                     np.array([0, 299, 150]))):
        if srcs is None:
            srcs = gg.pick_sources(g, 70, 5)
        dg = B.DeviceGraph.from_graph(g)
        _, st = B.bfs_multi(dg, srcs, flags=B.F_LEVEL_TIMING)
        k = st["num_levels"]
        assert k > 0
        assert np.all(st["ms"][:k] > 0) and np.all(st["ms_main"][:k] > 0)
        assert np.all(st["ms_main"][:k] <= st["ms"][:k] + 1e-3)
        assert float(st["ms"][:k].sum()) <= st["elapsed_ms"] + 1e-3


def _split_graphs():
    yield "rmat12", gg.rmat(12, seed=77), None
    yield "rmat14", gg.workload("rmat14"), None
    yield "directed", gg.directed_random(3000, 15000, seed=4, self_loops=True, duplicates=True), \
        np.arange(0, 3000, 47)[:64]
    yield "lattice", gg.lattice(90, seed=3), None
    yield "isolated", gg.from_edge_list(5, [(1, 2)], True), np.array([0, 1, 4])
    rng = np.random.default_rng(11)
    n = 9000
    src = np.concatenate([rng.integers(0, n, 30000), np.full(3000, 7), rng.integers(0, n, 2600)])
    dst = np.concatenate([rng.integers(0, n, 30000), rng.integers(0, n, 3000), np.full(2600, 4242)])
    yield "directed_hubs", gg.from_edge_list(n, np.stack([src, dst], 1), False), np.array([7, 4242, 1, 2, 3, 100])


@pytest.mark.parametrize("variant", [B.AUTO_HEURISTIC, B.PULL_B])
def test_forced_split_any_id(variant):
    """Split bottom-up levels (options.hub_split = T: in-edges from vertices
    below T pulled, frontier vertices at or above T pushed) give the oracle's
    depths for every T, and every bottom-up level is split.  On a split level
    the push expands exactly the frontier vertices >= T and examines all
    their out-edges (counts from the oracle's depths)."""
    for name, g, srcs in _split_graphs():
        g.with_csc()
        for v in range(g.n):  # the split needs ascending in-edge lists
            assert np.all(np.diff(g.csc_idx[g.csc_ptr[v]:g.csc_ptr[v + 1]]) >= 0)
        if srcs is None:
            srcs = gg.pick_sources(g, 64, 5)
        ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
        deg = np.diff(g.row_ptr.astype(np.int64))
        dg = B.DeviceGraph.from_graph(g)
        for t in sorted({1, 63, 64, 65, g.n // 3, max(g.n - 1, 1), g.n, g.n + 7}):
            lv, st = B.bfs_multi(dg, srcs, variant=variant, level_stats=True, hub_split=t)
            np.testing.assert_array_equal(lv.cpu().numpy(), ref, err_msg=f"{name} T={t} mode {variant}")
            k = st["num_levels"]
            assert k == int(ref.max()) + 1
            var = st["variant"][:k]
            assert not np.any(var == B.PULL_B), (name, t)
            if variant == B.PULL_B:
                assert np.all(var == B.MS_SPLIT), (name, t)
            tt = min(t, g.n)
            for lev in range(k):
                if var[lev] == B.MS_SPLIT:
                    front = (ref == lev).any(axis=0)
                    front[:tt] = False
                    assert int(st["push_sources"][lev]) == int(front.sum()), (name, t, lev)
                    assert int(st["scanned_push"][lev]) == int(deg[front].sum()), (name, t, lev)
                    assert int(st["scanned_push"][lev]) <= int(st["scanned"][lev])
                else:
                    assert int(st["scanned_push"][lev]) == 0 and int(st["push_sources"][lev]) == 0


def test_split_never_and_default_unsplit():
    """hub_split < 0 never splits; the default splits only graphs marked as
    numbered by degree (the input order here is not)."""
    g = gg.workload("rmat14")
    srcs = gg.pick_sources(g, 64, 5)
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    dg = B.DeviceGraph.from_graph(g)
    for hs in (-1, 0):
        lv, st = B.bfs_multi(dg, srcs, variant=B.PULL_B, level_stats=True, hub_split=hs)
        np.testing.assert_array_equal(lv.cpu().numpy(), ref)
        assert np.all(st["variant"][:st["num_levels"]] == B.PULL_B)


def test_main_timing_only():
    """BFS_F_MAIN_TIMING: each level's main kernel is timed (level_ms_main),
    the level's whole step is not (level_ms stays 0); depths unchanged."""
    g = gg.workload("rmat14")
    srcs = gg.pick_sources(g, 64, 5)
    dg = B.DeviceGraph.from_graph(g)
    lv, st = B.bfs_multi(dg, srcs, flags=B.F_MAIN_TIMING)
    k = st["num_levels"]
    assert k > 0
    assert np.all(st["ms_main"][:k] > 0) and np.all(st["ms"][:k] == 0)
    assert float(st["ms_main"][:k].sum()) <= st["elapsed_ms"] + 1e-3
    np.testing.assert_array_equal(lv.cpu().numpy(), oracle.multi(g.row_ptr, g.col_idx, srcs))


@pytest.mark.parametrize("variant", MODES)
def test_heavy_chunks_beyond_owner_table(variant):
    """More 1024-edge chunks of heavy vertices than the chunk-to-owner table
    holds (2n + 1024 entries): the later chunks find their vertex by search.
    A 48-vertex directed graph with duplicate edges (about 43K in- and
    out-edges on each of 40 vertices, about 1700 chunks per direction), and a
    path through the other 8."""
    rng = np.random.default_rng(21)
    n = 48
    m = 2_500_000
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    # vertices 40..47 only on a path 39 -> 40 -> ... -> 47, so depths grow past 2
    keep = (src < 40) & (dst < 40)
    src, dst = src[keep], dst[keep]
    path = np.array([[i, i + 1] for i in range(39, 47)])
    e = np.concatenate([np.stack([src, dst], 1), path])
    g = gg.from_edge_list(n, e, False)
    hchunks = int(np.sum(np.where(np.diff(g.csc_ptr) > 2048, (np.diff(g.csc_ptr) + 1023) // 1024, 0)))
    assert hchunks > 2 * n + 1024
    _check(g, np.array([0, 5, 39, 40, 47, 3, 3]), variant, level_stats=True)


@pytest.mark.parametrize("name", ["lattice4096", "er24"])
def test_full_size_every_row(name):
    """The lattice (4096^2, 10% of edges deleted, 0.1% shortcuts) and ER (2^24
    vertices, mean degree 8) configurations with their 32 sources, as
    generated: every row equal to the oracle (one search per host thread);
    and one single-source search (direction heuristic) against the oracle."""
    g = gg.workload(name)
    nsrc, sseed = gg.WORKLOAD_SOURCES[name]
    srcs = gg.pick_sources(g, nsrc, sseed)
    dg = B.DeviceGraph.from_graph(g)
    lv, st = B.bfs_multi(dg, srcs)
    got = lv.cpu().numpy()
    del lv
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    for i in range(nsrc):
        np.testing.assert_array_equal(got[i], ref[i], err_msg=f"{name} row {i}")
    lv1, _ = B.bfs_levels(dg, int(srcs[1]))
    np.testing.assert_array_equal(lv1.cpu().numpy(), ref[1], err_msg=f"{name} single")
