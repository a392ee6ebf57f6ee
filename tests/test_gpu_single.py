"""GPU parity of single-source BFS: every variant, every choice mode, against
the CPU oracle (depths bit-exact; parents by the Graph500-style check)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import checks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_17106_amd as B  # noqa: E402

VARIANTS = list(range(B.NUM_VARIANTS))


def _run(dg, g, s, variant, **kw):
    lv, par, st = B.bfs_parents(dg, int(s), variant=variant, **kw)
    return lv.cpu().numpy(), par.cpu().numpy(), st


def _check(g, s, lv, par, tag=""):
    ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
    np.testing.assert_array_equal(lv, ref, err_msg=f"depths differ {tag}")
    err = checks.check_parents(g.row_ptr, g.col_idx, int(s), lv, par)
    assert err is None, f"{tag}: {err}"
    return nl


def _tiny_graphs():
    out = []
    out.append(("path", gg.from_edge_list(7, [(i, i + 1) for i in range(6)], True)))
    out.append(("single", gg.from_edge_list(1, [], True)))
    out.append(("isolated_source", gg.from_edge_list(5, [(1, 2), (2, 3)], True)))
    out.append(("self_loops_dups", gg.from_edge_list(6, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 2), (2, 5)], True)))
    out.append(("directed_cycle", gg.from_edge_list(70, [(i, (i + 1) % 70) for i in range(70)], False)))
    out.append(("star_hub", gg.from_edge_list(5000, [(0, i) for i in range(1, 5000)], True)))
    out.append(("two_hubs", gg.from_edge_list(9000, [(0, i) for i in range(1, 4500)] +
                                              [(4500, i) for i in range(4501, 9000)] + [(1, 4501)], True)))
    for seed in range(3):
        out.append((f"dir{seed}", gg.directed_random(300 + 37 * seed, 1200, seed=seed, self_loops=True,
                                                     duplicates=True)))
    return out


@pytest.mark.parametrize("variant", VARIANTS)
def test_tiny_graphs_every_variant(variant):
    for name, g in _tiny_graphs():
        g.with_csc()
        dg = B.DeviceGraph.from_graph(g)
        for s in sorted({0, g.n - 1, g.n // 2}):
            lv, par, st = _run(dg, g, s, variant, level_stats=True)
            nl = _check(g, s, lv, par, f"{name} s={s} v={variant}")
            assert st["num_levels"] == nl
            assert st["reached"] == int((lv >= 0).sum())
            assert st["component_edges"] == oracle.edges_in_component(g.row_ptr, lv)


@pytest.mark.parametrize("variant", VARIANTS + [B.AUTO_HEURISTIC])
def test_rmat14_every_variant(variant):
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    srcs = gg.pick_sources(g, 4, 1402)
    for s in srcs:
        lv, par, _ = _run(dg, g, s, variant)
        _check(g, s, lv, par, f"rmat14 s={s} v={variant}")
        # levels-only entry point agrees too
        lv2, _ = B.bfs_levels(dg, int(s), variant=variant)
        np.testing.assert_array_equal(lv2.cpu().numpy(), lv)


def test_rmat22_every_fixed_variant():
    """The fixed-variant sweep's graph (R-MAT scale 22, 128M CSR entries):
    each fixed variant (and the two automatic modes) from three of its 64
    sources, depths equal to the oracle and parents valid -- the size where
    hub splitting, chunked temporary lists and large offsets are exercised."""
    g = gg.workload("rmat22")
    nsrc, sseed = gg.WORKLOAD_SOURCES["rmat22"]
    srcs = gg.pick_sources(g, nsrc, sseed)[[0, 31, 63]]
    ref = oracle.multi(g.row_ptr, g.col_idx, srcs)
    keys = checks.edge_keys(g.row_ptr, g.col_idx)
    dg = B.DeviceGraph.from_graph(g)
    for variant in VARIANTS + [B.AUTO_HEURISTIC, B.AUTO_LEARNED]:
        for i, s in enumerate(srcs):
            lv, par, _ = _run(dg, g, s, variant)
            np.testing.assert_array_equal(lv, ref[i], err_msg=f"rmat22 s={s} v={variant}")
            err = checks.check_parents(g.row_ptr, g.col_idx, int(s), lv, par, keys=keys)
            assert err is None, f"rmat22 s={s} v={variant}: {err}"


def test_level_stats_match_oracle_profile():
    g = gg.workload("rmat14").with_csc()
    dg = B.DeviceGraph.from_graph(g)
    (s,) = gg.pick_sources(g, 1, 1402)
    ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
    prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, ref)
    deg = g.out_degree()
    ld = np.floor(np.log2(1 + deg)).astype(np.int64)
    for variant in (B.PUSH_Q_BLOCK, B.PULL_B, B.AUTO_HEURISTIC):
        _, _, st = _run(dg, g, s, variant, level_stats=True)
        assert st["num_levels"] == nl
        np.testing.assert_array_equal(st["frontier"], prof["nF"])
        np.testing.assert_array_equal(st["frontier_edges"], prof["eF"])
        np.testing.assert_array_equal(st["unvisited"], prof["nU"])
        np.testing.assert_array_equal(st["unvisited_edges"], prof["eU"])
        for k in range(nl):
            assert st["frontier_ld"][k] == ld[ref == k].sum()
            assert st["frontier_ld2"][k] == (ld[ref == k] ** 2).sum()


def test_heuristic_decisions_match_replay():
    from oracle import heuristic
    g = gg.rmat(16, seed=4016).with_csc()
    dg = B.DeviceGraph.from_graph(g)
    for s in gg.pick_sources(g, 3, 77):
        ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
        prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, ref)
        lv, _, st = _run(dg, g, s, B.AUTO_HEURISTIC, level_stats=True)
        np.testing.assert_array_equal(lv, ref)
        dirs = heuristic.replay(g.n, prof["nF"], prof["eF"], prof["eU"])
        got = [1 if v == B.PULL_B else 0 for v in st["variant"]]
        assert got == dirs
        assert 1 in got  # the rule does switch on R-MAT


def test_random_schedules_give_identical_levels():
    rng = np.random.default_rng(11)
    for g in (gg.workload("rmat14"), gg.directed_random(4000, 30000, seed=5), gg.lattice(64, seed=2)):
        g.with_csc()
        dg = B.DeviceGraph.from_graph(g)
        for s in gg.pick_sources(g, 2, 3):
            ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
            for _ in range(6):
                sched = rng.integers(0, B.NUM_VARIANTS, size=nl + 1)
                lv, par, st = _run(dg, g, s, B.SCHEDULE, schedule=sched, level_stats=True)
                np.testing.assert_array_equal(lv, ref)
                assert checks.check_parents(g.row_ptr, g.col_idx, int(s), lv, par) is None
                np.testing.assert_array_equal(st["variant"], sched[:nl])


@pytest.mark.parametrize("variant", VARIANTS + [B.AUTO_HEURISTIC])
def test_lattice_and_er(variant):
    for g in (gg.lattice(300, seed=7), gg.erdos_renyi(1 << 15, 8.0, seed=8)):
        dg = B.DeviceGraph.from_graph(g)
        (s,) = gg.pick_sources(g, 1, 5)
        lv, par, _ = _run(dg, g, s, variant)
        _check(g, s, lv, par, f"{g.name} v={variant}")


def test_workspace_reuse_and_explicit_workspace():
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    ws = torch.empty(B.workspace_size(g.n), dtype=torch.uint8, device="cuda")
    for s in gg.pick_sources(g, 3, 9):
        lv, par, _ = B.bfs_parents(dg, int(s), variant=B.PUSH_Q_MERGE, workspace=ws)
        _check(g, s, lv.cpu().numpy(), par.cpu().numpy())


def test_error_codes():
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dg, -1)
    assert e.value.code == -1
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dg, g.n)
    assert e.value.code == -1
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dg, 0, workspace=small)
    assert e.value.code == -3
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dg, 0, variant=99)
    assert e.value.code == -1
    # pull without CSC
    dnc = B.DeviceGraph(g.n, g.row_ptr, g.col_idx)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dnc, 0, variant=B.PULL_B)
    assert e.value.code == -7
    # heuristic without CSC stays top-down and is still exact
    (s,) = gg.pick_sources(g, 1, 1402)
    lv, st = B.bfs_levels(dnc, int(s), variant=B.AUTO_HEURISTIC, level_stats=True)
    np.testing.assert_array_equal(lv.cpu().numpy(), oracle.bfs(g.row_ptr, g.col_idx, int(s))[0])
    assert (st["variant"] != B.PULL_B).all()
    # malformed CSR with validation on
    bad_col = g.col_idx.copy()
    bad_col[5] = g.n + 3
    dbad = B.DeviceGraph(g.n, g.row_ptr, bad_col)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dbad, 0, variant=B.PUSH_Q_BLOCK, flags=B.F_VALIDATE)
    assert e.value.code == -2
    bad_rp = g.row_ptr.copy()
    bad_rp[10], bad_rp[11] = bad_rp[11], bad_rp[10] - 1
    dbad = B.DeviceGraph(g.n, bad_rp, g.col_idx)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dbad, 0, variant=B.PUSH_Q_BLOCK, flags=B.F_VALIDATE)
    assert e.value.code == -2
    # level cap
    path = gg.from_edge_list(50, [(i, i + 1) for i in range(49)], True)
    dp = B.DeviceGraph.from_graph(path)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dp, 0, variant=B.PUSH_Q_BLOCK, max_levels=10)
    assert e.value.code == -6
    # learned strict mode without weights
    B.selector_clear()
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dg, 0, variant=B.AUTO_LEARNED, flags=B.F_STRICT_SELECTOR)
    assert e.value.code == -5
    lv, st = B.bfs_levels(dg, int(s), variant=B.AUTO_LEARNED)
    assert st["fell_back"] == 1
    np.testing.assert_array_equal(lv.cpu().numpy(), oracle.bfs(g.row_ptr, g.col_idx, int(s))[0])


@pytest.mark.parametrize("variant", [B.PULL_B, B.PULL_VIS])
def test_pull_scan_length_and_first_parent(variant):
    """Bottom-up steps examine exactly the sequential early-exit scan length
    (oracle eScan) and pick the first frontier in-neighbour in CSC order; with
    the visited set as the frontier (every visited in-neighbour of an
    unvisited vertex lies at the current depth) the result is the same."""
    for g in (gg.workload("rmat14"), gg.directed_random(3000, 40000, seed=12)):
        g.with_csc()
        dg = B.DeviceGraph.from_graph(g)
        (s,) = gg.pick_sources(g, 1, 21)
        ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
        prof = oracle.level_profile(g.row_ptr, g.csc_ptr, g.csc_idx, ref)
        lv, par, st = _run(dg, g, s, variant, level_stats=True)
        np.testing.assert_array_equal(lv, ref)
        np.testing.assert_array_equal(st["scanned"], prof["eScan"])
        for v in np.nonzero(ref > 0)[0][:2000]:
            ins = g.csc_idx[g.csc_ptr[v]:g.csc_ptr[v + 1]]
            first = ins[ref[ins] == ref[v] - 1][0]
            assert par[v] == first


def test_push_scanned_equals_frontier_edges():
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    (s,) = gg.pick_sources(g, 1, 1402)
    for v in (B.PUSH_Q_THREAD, B.PUSH_Q_BLOCK, B.PUSH_Q_MERGE, B.PUSH_B_ATOMIC, B.PUSH_B_NOATOMIC, B.PUSH_P3,
              B.PUSH_Q_FILTER, B.PUSH_B_FILTER, B.PUSH_Q_DEDUP):
        _, _, st = _run(dg, g, s, v, level_stats=True)
        np.testing.assert_array_equal(st["scanned"], st["frontier_edges"])
        np.testing.assert_array_equal(st["next"][:-1], st["frontier"][1:])
        assert st["next"][-1] == 0


@pytest.mark.parametrize("variant", VARIANTS + [B.AUTO_HEURISTIC])
def test_device_loop_every_variant(variant):
    """Levels enqueued ahead with device-side gating give the same depths,
    statistics and (heuristic) decisions as the host-driven loop."""
    for g in (gg.workload("rmat14"), gg.lattice(200, seed=6), gg.directed_random(2000, 9000, seed=2)):
        g.with_csc()
        dg = B.DeviceGraph.from_graph(g)
        for s in gg.pick_sources(g, 2, 4):
            lv, par, st = _run(dg, g, s, variant, flags=B.F_DEVICE_LOOP, level_stats=True)
            nl = _check(g, s, lv, par, f"device loop {g.name} v={variant}")
            _, _, st_h = _run(dg, g, s, variant, level_stats=True)
            assert st["num_levels"] == nl == st_h["num_levels"]
            for key in ("variant", "frontier", "frontier_edges", "unvisited", "unvisited_edges", "next"):
                np.testing.assert_array_equal(st[key], st_h[key], err_msg=key)
            if variant in (B.PULL_B, B.PULL_VIS):
                np.testing.assert_array_equal(st["scanned"], st_h["scanned"])
            assert st["host_syncs"] <= 1 + nl // 16 + 1


def test_device_loop_schedule_and_cap():
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    (s,) = gg.pick_sources(g, 1, 1402)
    ref, _, nl = oracle.bfs(g.row_ptr, g.col_idx, int(s))
    rng = np.random.default_rng(5)
    for _ in range(4):
        sched = rng.integers(0, B.NUM_VARIANTS, size=nl + 3)
        lv, par, st = _run(dg, g, s, B.SCHEDULE, schedule=sched, flags=B.F_DEVICE_LOOP, level_stats=True)
        np.testing.assert_array_equal(lv, ref)
        np.testing.assert_array_equal(st["variant"], sched[:nl])
    path = gg.from_edge_list(50, [(i, i + 1) for i in range(49)], True)
    dp = B.DeviceGraph.from_graph(path)
    with pytest.raises(B.BfsError) as e:
        B.bfs_levels(dp, 0, variant=B.PUSH_Q_BLOCK, max_levels=10, flags=B.F_DEVICE_LOOP)
    assert e.value.code == -6
    lv, st = B.bfs_levels(dp, 0, variant=B.AUTO_HEURISTIC, flags=B.F_DEVICE_LOOP)
    np.testing.assert_array_equal(lv.cpu().numpy(), np.arange(50))
    assert st["num_levels"] == 50


def test_device_loop_timing_fills_level_ms():
    g = gg.workload("rmat14")
    dg = B.DeviceGraph.from_graph(g)
    (s,) = gg.pick_sources(g, 1, 1402)
    for fl in (0, B.F_DEVICE_LOOP):
        _, st = B.bfs_levels(dg, int(s), variant=B.AUTO_HEURISTIC, flags=B.F_LEVEL_TIMING | fl)
        assert (st["ms"] > 0).all() and len(st["ms"]) == st["num_levels"]


@pytest.mark.parametrize("variant", [B.PUSH_Q_FILTER, B.PUSH_B_FILTER])
def test_filter_variant_many_chunks(variant):
    """Advance then filter with frontiers whose edges fill the temporary list
    many times over (R-MAT 16: 65,536 entries against levels of ~1.5M edges),
    host loop and device loop; scanned edges are the frontier's out-edges."""
    g = gg.rmat(16, seed=1616)
    dg = B.DeviceGraph.from_graph(g)
    (s,) = gg.pick_sources(g, 1, 17)
    for flags in (0, B.F_DEVICE_LOOP):
        lv, par, st = _run(dg, g, s, variant, flags=flags, level_stats=True)
        _check(g, s, lv, par, f"flags {flags}")
        assert int(st["frontier_edges"].max()) > 8 * 65536
        np.testing.assert_array_equal(st["scanned"], st["frontier_edges"])


def test_dedup_variant_list_overflow():
    """Best-effort deduplication (Table 3, variant 9).  A complete bipartite
    level (source -> 300 vertices -> the same 300 others) makes 90,000
    candidates, duplicates across waves, against a temporary list of 65,536
    entries, so the candidates past the list are claimed in the advance;
    R-MAT 16 is the ordinary case.  Host loop and device loop, and mixed into
    random schedules with bitmap consumers (pull, bitmap push)."""
    a_side = list(range(1, 301))
    b_side = list(range(301, 601))
    e = [(0, x) for x in a_side] + [(x, y) for x in a_side for y in b_side] + [(600, 601), (601, 602)]
    bip = gg.from_edge_list(603, e, True)
    r16 = gg.rmat(16, seed=1616)
    for g, (s,) in ((bip, (0,)), (r16, gg.pick_sources(r16, 1, 17))):
        dg = B.DeviceGraph.from_graph(g)
        for flags in (0, B.F_DEVICE_LOOP):
            lv, par, st = _run(dg, g, s, B.PUSH_Q_DEDUP, flags=flags, level_stats=True)
            _check(g, s, lv, par, f"{g.name} flags {flags}")
            np.testing.assert_array_equal(st["scanned"], st["frontier_edges"])
            np.testing.assert_array_equal(st["next"][:-1], st["frontier"][1:])
        rng = np.random.default_rng(9)
        for _ in range(4):
            sched = rng.choice([B.PUSH_Q_DEDUP, B.PULL_B, B.PUSH_B_ATOMIC, B.PUSH_Q_DEDUP, B.PUSH_P3], 12).tolist()
            lv, par, _ = _run(dg, g, s, B.SCHEDULE, schedule=sched)
            _check(g, s, lv, par, f"{g.name} schedule {sched}")
    assert int(np.diff(bip.row_ptr)[1:301].sum()) - 300 > 65536  # the bipartite level overflows the list
