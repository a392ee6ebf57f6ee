#!/usr/bin/env python3
"""BFS throughput on one MI355X: GTEPS and HBM-roofline fraction.

Workload: R-MAT scale 22 (4,194,304 vertices, edge factor 16, a,b,c,d =
.57,.19,.19,.05, seeded relabel, symmetrised, self-loops and duplicate edges
removed; 128,307,516 CSR entries) and 64 seeded sources from its largest
component.  One step = the depths from all 64 sources, computed by the
64-lane bit-packed multi-source search (bfs_multi) -- the batched form of this
job -- on the graph renumbered by decreasing out-degree (bfs_reorder_degree,
a preprocessing step like the paper's own renumbering of every graph; its
time is reported as config.reorder_ms), with sources and depths in the
original numbering (options.vertex_map).  The same search on the graph as
generated is reported as input_order, and on the graph renumbered by reverse
Cuthill-McKee (the paper's own preprocessing) as rcm_order.  Inputs are resident in HBM before the
timed region.  The same JSON line
also reports, on the same graph and sources, the single-source forms (learned
per-level selector, direction heuristic, every fixed variant) and the
512-instance batched launch against instance-by-instance runs.

  python bench.py [--steps K] [--warmup W] [--no-sweep] [--no-batch]

GTEPS counts undirected edges of the traversed component: (sum of
out-degrees of reached vertices) / 2, summed over sources.  The roofline
block prices the dominant kernel (the step type with the most time in the
timed region) with the algorithmic byte model of
paper_2607_17106_amd.bytemodel; its time comes from HIP events the library
records on the stream it launches on, inside the timed region.  It also
gives the rate of a plain 1 GiB device copy on the same device (copy_gbs).
cpu_baseline is the oracle on the host: one instance per thread (value) and
one thread alone (single_thread).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of k_ms_pull_tile on this workload: two rocprofv3 --pmc runs of
# `bench.py --steps 3 --warmup 1 --no-sweep --no-batch --no-cpu --no-input-order
# --multi-config <configuration>` (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch averaged over the kernel's 28 dispatches: 7 steps of 4 bottom-up
# levels), each scaled by what the same counter reads for a plain copy of
# 1 GiB (`bench.py --copy-calibration 1073741824`: FETCH_SIZE 524300 KiB ->
# x2.0, WRITE_SIZE 1048576 KiB -> x1.0), for each configuration the autotuner
# has been seen to choose (its choice between near-equal ones varies from run
# to run).  Reported only while the kernel code (comments and whitespace
# aside) hashes to the values the counters were taken with and the steps run
# with one of these configurations.
TILE_TRAFFIC = {
    "sources_sha256": {
        "paper_2607_17106_amd/csrc/msbfs.hip": "29dce350f2e83ce93803c984dec46e9e83d7871ec32335b0faa6e299e413f868",
        "paper_2607_17106_amd/csrc/common.hpp": "f27b9929ec1714fbf3159a3009a7159008f386ef7997698178ca13137ff29019",
    },
    "records": [
        {"multi_config": {"wide_ratio": 16, "split_vpt": 4, "cap0": 32, "tile_alpha": 64, "alpha": 7, "split_lout": 16,
                          "wide_vpt": 2, "narrow_vpt": 4},
         "fetch_kib": 181835.6, "write_kib": 107162.0},
        {"multi_config": {"wide_ratio": 16, "split_vpt": 4, "cap0": 32, "tile_alpha": 64, "alpha": 7, "split_lout": 16,
                          "wide_vpt": 1, "narrow_vpt": 4},
         "fetch_kib": 183245.8, "write_kib": 107341.6},
        {"multi_config": {"wide_ratio": 8, "split_vpt": 4, "cap0": 32, "tile_alpha": 64, "alpha": 7, "split_lout": 16,
                          "wide_vpt": 2, "narrow_vpt": 4},
         "fetch_kib": 181857.3, "write_kib": 107162.1},
    ],
    "fetch_scale": 2.0, "write_scale": 1.0,
}

# The same for k_batch on the 512-instance mix: `bench.py --steps 1 --warmup 1
# --no-sweep --no-cpu --no-input-order --multi-config ...` (the autotuner's
# candidate runs, then the warm-up and timed call of the chosen configuration
# below, whose two dispatches are averaged), with the copy calibration above.
BATCH_TRAFFIC = {
    "sources_sha256": {
        "paper_2607_17106_amd/csrc/batch.hip": "af1d9fdfa27cd3723a8cdc8d0c412198d82116584f8e5573d8b2f5c5d515e7fe",
        "paper_2607_17106_amd/csrc/common.hpp": "f27b9929ec1714fbf3159a3009a7159008f386ef7997698178ca13137ff29019",
    },
    "config": {"block_threads": 1024, "blocks_per_cu": 2, "small_vertices": 1048576, "team_vertices": 131072,
               "max_team": 8},
    "fetch_kib": 11435993.5, "write_kib": 4903784.0, "fetch_scale": 2.0, "write_scale": 1.0,
}


def code_hash(path: str) -> str:
    """sha256 of a C/HIP source with comments and whitespace removed, so that
    only code changes count."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256("".join(text.split()).encode()).hexdigest()


def measured_traffic_bytes(t: dict, config_key: str, config: dict):
    """Measured HBM bytes per launch from the record t, or None once the
    kernel code differs from the code the counters were taken with, or the
    run uses another configuration."""
    for rel, h in t["sources_sha256"].items():
        if code_hash(os.path.join(ROOT, rel)) != h:
            return None
    for rec in t.get("records", [t]):
        if rec.get(config_key) == config:
            return (rec["fetch_kib"] * t["fetch_scale"] + rec["write_kib"] * t["write_scale"]) * 1024.0
    return None
METRIC = "GTEPS and HBM-roofline fraction at 1 GPU: fixed variant vs learned/batched"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_cores() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS where that is set (the share of a shared host)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(cap))) if cap.isdigit() and int(cap) > 0 else n


def cpu_baseline(g, sources, seconds: float):
    """The oracle (plain FIFO-queue BFS in C) on a bounded sample of the same
    sources.  Single thread: whole searches until `seconds` of BFS time.  All
    cores: one oracle search per thread at a time (the C call releases the
    GIL), thread t taking sources t, t+T, t+2T, ... (wrapping), until
    `seconds`/2 of wall time; throughput = edges of the searches finished in
    that wall time / that wall time.  `value` is the all-core figure."""
    import threading
    import numpy as np
    import oracle  # the CPU oracle is used here only, as the reported baseline
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    deg = np.diff(rp.astype(np.int64))
    edges = 0
    dt = 0.0
    done = 0
    for s in sources:
        t0 = time.perf_counter()
        lv, _, _ = oracle.bfs(rp, ci, int(s), want_parents=False)
        dt += time.perf_counter() - t0
        edges += int(deg[lv >= 0].sum()) // 2
        done += 1
        if dt >= seconds:
            break
    single = round(edges / dt / 1e9, 4)

    cores = cpu_cores()
    wall = max(seconds / 2, 2.0)
    res = [[0, 0] for _ in range(cores)]
    t_start = time.perf_counter()

    def worker(t):
        i = t
        while time.perf_counter() - t_start < wall:
            lv, _, _ = oracle.bfs(rp, ci, int(sources[i % len(sources)]), want_parents=False)
            res[t][0] += int(deg[lv >= 0].sum()) // 2
            res[t][1] += 1
            i += cores
    th = [threading.Thread(target=worker, args=(t,)) for t in range(cores)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    wall_all = time.perf_counter() - t_start
    e_all = sum(r[0] for r in res)
    n_all = sum(r[1] for r in res)
    return {"value": round(e_all / wall_all / 1e9, 4), "unit": "GTEPS", "cores": cores, "kind": "oracle",
            "sample": f"all cores: {n_all} single-source searches of the same graph and sources, one oracle "
                      f"instance per thread, {wall_all:.1f} s wall; single thread: {done} of {len(sources)} "
                      f"searches, {dt:.1f} s of BFS time; {cpu_model()}",
            "single_thread": {"value": single, "unit": "GTEPS", "cores": 1}}


def copy_rate_gbs(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Bytes read plus bytes written per second by a plain device-to-device
    copy of `nbytes` (torch's copy kernel), timed with events: the HBM rate a
    streaming kernel reaches on this part, for scale beside the published peak."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del src, dst
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip single-source modes and fixed variants")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-instance batch")
    ap.add_argument("--sweep-sources", type=int, default=16)
    ap.add_argument("--roofline-sources", type=int, default=4,
                    help="sources per mode for the single-source per-variant roofline (level-timed searches)")
    ap.add_argument("--multi-config", default=None, metavar="JSON",
                    help="bfs_multi_config fields for the 64-lane steps instead of autotuning (as the "
                         "counter runs use, so every profiled step has the same configuration); the "
                         "library-defaults comparison is then skipped")
    ap.add_argument("--no-input-order", action="store_true",
                    help="skip the comparison runs on the graph as generated and renumbered by RCM "
                         "(profiles see the timed step only)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times): the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the search runs on one "
              "device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}))
        return
    import numpy as np
    import graphgen as gg
    import paper_2607_17106_amd as B
    from paper_2607_17106_amd import bytemodel, selector

    torch.cuda.set_device(0)
    t0 = time.time()
    g = gg.workload(args.workload)
    nsrc, sseed = gg.WORKLOAD_SOURCES.get(args.workload, (args.sources, 1))
    sources = gg.pick_sources(g, min(args.sources, nsrc), sseed)
    log(f"[bench] graph {g.name}: n={g.n} nnz={g.nnz} sources={len(sources)} ({time.time() - t0:.1f} s)")
    dg = B.DeviceGraph.from_graph(g)
    lv_multi = torch.empty((len(sources), g.n), dtype=torch.int32, device="cuda")
    ws_multi = torch.empty(B.workspace_size(g.n, 64), dtype=torch.uint8, device="cuda")
    # preprocessing: renumbering by decreasing out-degree (second call timed)
    B.reorder_degree(dg)
    (rg, new_of_old, _), reorder_s = timed(lambda: B.reorder_degree(dg))
    log(f"[bench] renumbered by out-degree in {reorder_s * 1e3:.1f} ms")

    # ---------------------------------------------------------- timed step
    # timing: 0 none, 1 the main kernel of each level (HIP events around it:
    # the tile kernel's duration for the roofline), 2 every level's step too.
    # config None: the configuration bfs_multi_autotune stored for the graph.
    def step(timing, graph=rg, vmap=new_of_old, config=None):
        flags = (0, B.F_MAIN_TIMING, B.F_LEVEL_TIMING)[timing]
        return B.bfs_multi(graph, sources, flags=flags, workspace=ws_multi, levels=lv_multi, vertex_map=vmap,
                           config=config)[1]

    def autotune(graph, vmap):
        return timed(lambda: B.bfs_multi_autotune(graph, sources, workspace=ws_multi, levels=lv_multi,
                                                  vertex_map=vmap))

    # autotuning, like the renumbering, is per-graph preparation outside the
    # timed region; the defaults are timed too, after the tuned steps
    if args.multi_config:
        tuned, tune_s = B.MultiConfig(**json.loads(args.multi_config)), 0.0
        given = tuned

        def step(timing, graph=rg, vmap=new_of_old, config=None, _step=step):  # noqa: F811
            return _step(timing, graph, vmap, given if config is None else config)
        log(f"[bench] configuration given: {tuned}")
    else:
        (tuned, tuned_ms), tune_s = autotune(rg, new_of_old)
        log(f"[bench] autotuned in {tune_s:.2f} s: {tuned} ({tuned_ms:.3f} ms)")

    for _ in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        stats.append(step(1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"[bench] {args.steps} timed steps done in {elapsed * 1e3:.2f} ms")
    gteps = sum(st["component_edges"] for st in stats) / 2 / elapsed / 1e9
    # per-level step times for the diagnostics below, from the same steps run
    # again after the timed region
    stats_lev = [step(2) for _ in range(args.steps)]
    # the library defaults (no tuning), for comparison: the same steps with
    # the same main-kernel events
    default_ms = None
    if not args.multi_config:
        step(1, config=B.MultiConfig())
        torch.cuda.synchronize()
        t_d = time.perf_counter()
        for _ in range(args.steps):
            step(1, config=B.MultiConfig())
        torch.cuda.synchronize()
        default_ms = (time.perf_counter() - t_d) * 1e3 / args.steps
        log(f"[bench] library defaults: {default_ms:.3f} ms per step")

    # the same search on the graph as generated (no renumbering), for comparison
    input_order = rcm_order = None
    if not args.no_input_order and not args.multi_config:
        (tuned_in, _), tune_in_s = autotune(dg, None)
        step(0, dg, None)
        torch.cuda.synchronize()
        t_in = time.perf_counter()
        st_in = [step(0, dg, None) for _ in range(args.steps)]
        torch.cuda.synchronize()
        el_in = time.perf_counter() - t_in
        input_order = {"gteps": round(sum(st["component_edges"] for st in st_in) / 2 / el_in / 1e9, 3),
                       "ms_per_step": round(el_in * 1e3 / args.steps, 3), "multi_config": vars(tuned_in),
                       "autotune_s": round(tune_in_s, 2)}
        # the tile kernel's roofline on this graph, from steps run again with
        # the main-kernel events (outside the timed loop above)
        t_in = b_in = 0.0
        n_in = 0
        for st in [step(1, dg, None) for _ in range(args.steps)]:
            tb = bytemodel.ms_tile_level_bytes(st, g.n)
            for k in range(st["num_levels"]):
                if tb[k] is not None:
                    t_in += float(st["ms_main"][k])
                    b_in += tb[k]
                    n_in += 1
        a_in = b_in / (t_in * 1e-3) / 1e9
        input_order["roofline"] = {"bound": "hbm", "achieved": round(a_in, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(a_in / HBM_PEAK_GBS, 4), "traffic": None,
                                   "kernel": "k_ms_pull_tile", "launches": n_in,
                                   "avg_launch_us": round(t_in * 1e3 / max(n_in, 1), 2),
                                   "bytes_per_launch": round(b_in / max(n_in, 1))}
        log(f"[bench] input order: {input_order}")
        # and on the graph renumbered by reverse Cuthill-McKee
        (cg, cmap, _), rcm_s = timed(lambda: B.reorder_rcm(dg))
        if not args.multi_config:
            autotune(cg, cmap)
        step(0, cg, cmap)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        st_c = [step(0, cg, cmap) for _ in range(args.steps)]
        torch.cuda.synchronize()
        el_c = time.perf_counter() - t_c
        rcm_order = {"gteps": round(sum(st["component_edges"] for st in st_c) / 2 / el_c / 1e9, 3),
                     "ms_per_step": round(el_c * 1e3 / args.steps, 3), "reorder_ms": round(rcm_s * 1e3, 1)}
        log(f"[bench] rcm order: {rcm_order}")
        del cg, cmap

    # roofline of the dominant kernel: the bottom-up tile kernel (k_ms_pull_tile),
    # timed alone by the library's HIP events on its stream, priced by its own
    # algorithmic bytes (bytemodel.ms_tile_bytes)
    t_tile = b_tile = 0.0
    n_tile = 0
    per_t, per_b = {}, {}
    for st in stats:
        tb = bytemodel.ms_tile_level_bytes(st, g.n)
        for k in range(st["num_levels"]):
            if tb[k] is not None:
                t_tile += float(st["ms_main"][k])
                b_tile += tb[k]
                n_tile += 1
    tile_lev = 0.0
    for st in stats_lev:
        lb = bytemodel.ms_level_bytes(st, g.n)
        for k in range(st["num_levels"]):
            v = {B.PULL_B: "bottom_up_step", B.MS_SPLIT: "split_step"}.get(int(st["variant"][k]), "top_down_step")
            per_t[v] = per_t.get(v, 0.0) + float(st["ms"][k])
            per_b[v] = per_b.get(v, 0.0) + lb[k]
            if int(st["variant"][k]) in (B.PULL_B, B.MS_SPLIT):
                tile_lev += float(st["ms_main"][k])
    achieved = b_tile / (t_tile * 1e-3) / 1e9
    step_level_ms = sum(per_t.values()) / len(stats_lev)
    traffic = (measured_traffic_bytes(TILE_TRAFFIC, "multi_config", vars(tuned))
               if args.workload == "rmat22" and len(sources) == 64 else None)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic) if traffic is not None else None, "kernel": "k_ms_pull_tile",
            "launches": n_tile, "avg_launch_us": round(t_tile * 1e3 / max(n_tile, 1), 2),
            "bytes_per_launch": round(b_tile / max(n_tile, 1)),
            "time_share_of_level_steps": round(tile_lev / len(stats_lev) / step_level_ms, 3),
            "level_steps_gbs": {k: round(per_b[k] / (per_t[k] * 1e-3) / 1e9, 1) for k in per_t}}
    copy_gbs = copy_rate_gbs(torch)
    roof["copy_gbs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if traffic is not None:
        roof["traffic_over_algorithmic"] = round(traffic / (b_tile / max(n_tile, 1)), 2)
    st0 = stats_lev[0]
    for k in range(st0["num_levels"]):
        log(f"[bench] ms level {k}: {({B.PULL_B: 'pull', B.MS_SPLIT: 'split'}).get(int(st0['variant'][k]), 'push')} "
            f"active={st0['frontier'][k]} ef={st0['frontier_edges'][k]} eu={st0['unvisited_edges'][k]} "
            f"unvis={st0['unvisited'][k]} scan={st0['scanned'][k]} "
            f"new={st0['next'][k]} pushed={st0['scanned_push'][k]} ms={st0['ms'][k]:.4f}")
    out = {"metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"{args.workload}-{len(sources)}src", "graph": "R-MAT scale 22, edge factor 16, "
                      "a,b,c,d=.57,.19,.19,.05, symmetrised", "n": g.n, "nnz": g.nnz, "sources": len(sources),
                      "method": "64-lane bit-packed multi-source BFS (bfs_multi)", "output": "depths [64][n]",
                      "vertex_order": "renumbered by decreasing out-degree (bfs_reorder_degree, preprocessing, "
                                      "outside the timed region); sources and depths in the original numbering",
                      "reorder_ms": round(reorder_s * 1e3, 2), "multi_config": vars(tuned),
                      "autotune_s": round(tune_s, 2),
                      "library_defaults_ms_per_step": round(default_ms, 3) if default_ms is not None else None},
           "roofline": roof, "input_order": input_order, "rcm_order": rcm_order}

    # ------------------------------------------- single-source comparisons
    if not args.no_sweep:
        ws = torch.empty(B.workspace_size(g.n), dtype=torch.uint8, device="cuda")
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")

        def run_single(var, srcs, graph=dg, vmap=None):
            edges = 0
            for s in srcs:
                _, st = B.bfs_levels(graph, int(s), variant=var, workspace=ws, levels=lv, vertex_map=vmap)
                edges += st["component_edges"] // 2
            return edges

        single = {}
        have_learned = selector.load_default()
        modes = [("heuristic", B.AUTO_HEURISTIC, sources)]
        if have_learned:
            modes.insert(0, ("learned", B.AUTO_LEARNED, sources))
        modes += [(B.VARIANT_NAMES[v], v, sources[: args.sweep_sources]) for v in range(B.NUM_VARIANTS)]
        for name, var, srcs in modes:
            run_single(var, srcs[:2])  # warm-up
        # best of 3 passes over the sources, the modes taking turns within each
        # pass: a pass is a few ms of host-driven launches, and one host stall
        # of tens of ms would halve its rate
        best, edges_of = {}, {}
        for _ in range(3):
            for name, var, srcs in modes:
                edges_of[name], dt = timed(lambda: run_single(var, srcs))
                best[name] = min(best.get(name, dt), dt)
        for name, _, _ in modes:
            single[name] = round(edges_of[name] / best[name] / 1e9, 3)
            log(f"[bench] single-source {name}: {single[name]} GTEPS")
        # per-variant roofline: algorithmic bytes of every level step (the
        # byte model over the library's per-level counts) over the steps'
        # device time (HIP events around each level's kernels), on a few
        # level-timed searches per mode, outside the timed passes above
        roof_single = {}
        for name, var, srcs in modes:
            b_sum = t_sum = 0.0
            for s_ in srcs[: args.roofline_sources]:
                _, st = B.bfs_levels(dg, int(s_), variant=var, workspace=ws, levels=lv, flags=B.F_LEVEL_TIMING)
                b_sum += sum(bytemodel.level_bytes(st, g.n))
                t_sum += float(st["ms"][: st["num_levels"]].sum())
            gbs = b_sum / (t_sum * 1e-3) / 1e9
            roof_single[name] = {"achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                 "bytes_per_search": round(b_sum / max(1, min(len(srcs), args.roofline_sources))),
                                 "step_ms_per_search": round(t_sum / max(1, min(len(srcs), args.roofline_sources)), 4)}
        out["single_source_roofline"] = roof_single
        log(f"[bench] single-source roofline: { {k: v['frac'] for k, v in roof_single.items()} }")
        # the direction heuristic on the degree-renumbered graph (vertex_map)
        run_single(B.AUTO_HEURISTIC, sources[:2], rg, new_of_old)
        ren_t = None
        for _ in range(3):
            ren_e, dt = timed(lambda: run_single(B.AUTO_HEURISTIC, sources, rg, new_of_old))
            ren_t = dt if ren_t is None else min(ren_t, dt)
        out["single_source_renumbered_heuristic_gteps"] = round(ren_e / ren_t / 1e9, 3)
        log(f"[bench] single-source heuristic, renumbered graph: {out['single_source_renumbered_heuristic_gteps']} GTEPS")
        fixed = {k: v for k, v in single.items() if k not in ("learned", "heuristic")}
        best_fixed = max(fixed, key=fixed.get)
        out["single_source_gteps"] = single
        out["single_source_timing"] = ("wall clock, best of 3 passes; learned and heuristic over all "
                                       f"{len(sources)} sources, fixed variants over the first {args.sweep_sources}")
        out["best_fixed_variant"] = {"name": best_fixed, "gteps": fixed[best_fixed]}
        out["multi_vs_best_fixed"] = round(gteps / fixed[best_fixed], 2)
        if have_learned:
            out["learned_vs_best_fixed"] = round(single["learned"] / fixed[best_fixed], 2)
            out["learned_vs_heuristic"] = round(single["learned"] / single["heuristic"], 2)
        B.selector_clear()

    # ------------------------------------------------ 512-instance batch
    if not args.no_batch:
        t1 = time.time()
        bb = gg.mixed_batch(512, seed=5501)
        log(f"[bench] batch of {bb.num}: n={bb.total_n} nnz={bb.total_nnz} ({time.time() - t1:.0f} s)")
        db = B.DeviceBatch(bb)
        lvb = torch.empty(bb.total_n, dtype=torch.int32, device="cuda")
        cfg, tune_ms = B.bfs_batch_autotune(db, levels=lvb)
        B.bfs_batch(db, levels=lvb)
        (lvb, stb), dtb = timed(lambda: B.bfs_batch(db, levels=lvb))
        batch_gteps = stb["component_edges"] / 2 / dtb / 1e9
        # instance by instance with a fixed variant and with the heuristic, on every 8th instance
        sub = list(range(0, bb.num, 8))
        sub_batch = gg.concat([bb.graphs[i] for i in sub], [int(bb.sources[i]) for i in sub])
        dsub = B.DeviceBatch(sub_batch)
        lvs = torch.empty(sub_batch.total_n, dtype=torch.int32, device="cuda")
        B.bfs_batch(dsub, levels=lvs)
        (_, sts), dts = timed(lambda: B.bfs_batch(dsub, levels=lvs))
        dgs = [B.DeviceGraph.from_graph(bb.graphs[i]) for i in sub]
        one = {}
        for name, var in (("heuristic", B.AUTO_HEURISTIC), ("push_b_noatomic", B.PUSH_B_NOATOMIC)):
            def one_by_one():
                e = 0
                for d, i in zip(dgs, sub):
                    _, st = B.bfs_levels(d, int(bb.sources[i]), variant=var)
                    e += st["component_edges"] // 2
                return e
            one_by_one()
            e, dt = timed(one_by_one)
            one[name] = round(e / dt / 1e9, 3)
        # roofline of the batched kernel: its algorithmic bytes over the device
        # time of the call (HIP events around the state-clearing and search
        # kernels on the library's stream)
        reached = int((lvb >= 0).sum().item())
        bb_bytes = bytemodel.batch_bytes(bb.total_n, reached, int(stb["component_edges"]))
        b_ach = bb_bytes / (stb["elapsed_ms"] * 1e-3) / 1e9
        bcfg = {"block_threads": cfg.block_threads, "blocks_per_cu": cfg.blocks_per_cu,
                "small_vertices": cfg.small_vertices, "team_vertices": cfg.team_vertices, "max_team": cfg.max_team}
        # With no instance above small_vertices nothing is searched by a team:
        # configurations that differ only in the team fields launch the same
        # work, so the counters taken with one stand for the others.
        rec, bcmp = BATCH_TRAFFIC, bcfg
        team_keys = ("team_vertices", "max_team")
        if int(np.diff(bb.v_off).max()) <= cfg.small_vertices:
            rec = dict(rec, config={k: v for k, v in rec["config"].items() if k not in team_keys})
            bcmp = {k: v for k, v in bcfg.items() if k not in team_keys}
        b_traffic = measured_traffic_bytes(rec, "config", bcmp)
        b_roof = {"bound": "hbm", "achieved": round(b_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(b_ach / HBM_PEAK_GBS, 4),
                  "traffic": round(b_traffic) if b_traffic is not None else None,
                  "kernel": "k_batch", "bytes_per_launch": round(bb_bytes)}
        if b_traffic is not None:
            b_roof["traffic_over_algorithmic"] = round(b_traffic / bb_bytes, 2)
        out["batch512"] = {"gteps": round(batch_gteps, 3), "ms": round(dtb * 1e3, 2),
                           "kernel_ms": round(stb["elapsed_ms"], 3), "roofline": b_roof, "config": bcfg,
                           "autotune_best_ms": round(tune_ms, 2),
                           "sample_64_instances": {"batched_gteps": round(sts["component_edges"] / 2 / dts / 1e9, 3),
                                                   "one_by_one_gteps": one}}
        log(f"[bench] batch512 {out['batch512']}")
        del db, dsub, dgs

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, list(sources), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
