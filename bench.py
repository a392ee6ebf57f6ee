#!/usr/bin/env python3
"""BFS throughput on one MI355X: GTEPS and HBM-roofline fraction.

Workload: R-MAT scale 22 (4,194,304 vertices, edge factor 16, a,b,c,d =
.57,.19,.19,.05, symmetrised, self-loops and duplicates removed), 64 seeded
sources from the largest component.  One step = one BFS from each of the 64
sources with the per-level variant choice (learned selector when trained
weights are present, else the direction heuristic); depths only.  Inputs are
resident in HBM before the timed region.

  python bench.py [--steps K] [--warmup W] [--mode learned|heuristic|<variant>]

Prints ONE JSON line.  GTEPS counts undirected edges of the traversed
component: (sum of out-degrees of reached vertices) / 2, summed over sources.
The roofline block prices the dominant step kernel with the algorithmic byte
model of paper_2607_17106_amd.bytemodel, timed with HIP events on the stream
the library launches on, inside the timed region.
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


def cpu_baseline(g, sources, seconds: float):
    """The oracle (plain FIFO-queue BFS in C, one thread) on a bounded sample
    of the same sources: runs whole BFSs until `seconds` have elapsed."""
    import oracle  # the CPU oracle is used here only, as the reported baseline
    edges = 0
    dt = 0.0
    done = 0
    for s in sources:
        t0 = time.perf_counter()
        lv, _, _ = oracle.bfs(g.row_ptr, g.col_idx, int(s), want_parents=False)
        dt += time.perf_counter() - t0
        edges += oracle.edges_in_component(g.row_ptr, lv) // 2
        done += 1
        if dt >= seconds:
            break
    return {"value": round(edges / dt / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{done} of {len(sources)} sources, whole BFSs, {dt:.1f} s, {cpu_model()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--mode", default="auto")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the fixed-variant comparison")
    ap.add_argument("--sweep-sources", type=int, default=16)
    ap.add_argument("--device-loop", action="store_true",
                    help="persistent whole-search kernel instead of the host-driven level loop")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on more than one GPU are not part of this build "
              "(see DESIGN.md, 'Sharding')", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import graphgen as gg
    import paper_2607_17106_amd as B
    from paper_2607_17106_amd import bytemodel, selector

    torch.cuda.set_device(0)
    t0 = time.time()
    g = gg.workload(args.workload)
    nsrc, sseed = gg.WORKLOAD_SOURCES.get(args.workload, (args.sources, 1))
    sources = gg.pick_sources(g, min(args.sources, nsrc) if args.sources else nsrc, sseed)
    log(f"[bench] graph {g.name}: n={g.n} nnz={g.nnz} sources={len(sources)} ({time.time() - t0:.1f} s)")
    dg = B.DeviceGraph.from_graph(g)
    ws = torch.empty(B.workspace_size(g.n), dtype=torch.uint8, device="cuda")
    levels = torch.empty(g.n, dtype=torch.int32, device="cuda")

    mode = args.mode
    if mode == "auto":
        mode = "learned" if selector.load_default() else "heuristic"
    elif mode == "learned":
        if not selector.load_default():
            log("[bench] no trained selector weights found; learned mode falls back to the heuristic")
    variant = {"learned": B.AUTO_LEARNED, "heuristic": B.AUTO_HEURISTIC}.get(mode)
    if variant is None:
        inv = {v: k for k, v in B.VARIANT_NAMES.items()}
        variant = inv[mode]

    loop_flag = B.F_DEVICE_LOOP if args.device_loop else 0

    def one_pass(var, srcs, timing=True, events=None):
        flags = (B.F_LEVEL_TIMING if timing else 0) | loop_flag
        sts = []
        stream = torch.cuda.current_stream()
        for s in srcs:
            if events is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            _, st = B.bfs_levels(dg, int(s), variant=var, flags=flags, workspace=ws, levels=levels)
            if events is not None:
                e1.record(stream)
                events.append((e0, e1))
            sts.append(st)
        return sts

    for _ in range(args.warmup):
        one_pass(variant, sources, timing=False)
    torch.cuda.synchronize()
    all_stats = []
    call_events = []
    t_start = time.perf_counter()
    for step in range(args.steps):
        all_stats.extend(one_pass(variant, sources, events=call_events))
        log(f"[bench] step {step + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    teps_edges = sum(st["component_edges"] for st in all_stats) / 2
    gteps = teps_edges / elapsed / 1e9
    ms_per_step = elapsed * 1e3 / args.steps

    # roofline of the dominant kernel over the timed region
    per_var_t, per_var_b, per_var_n = {}, {}, {}
    for st in all_stats:
        bts = bytemodel.level_bytes(st, g.n)
        for k in range(st["num_levels"]):
            v = int(st["variant"][k])
            per_var_t[v] = per_var_t.get(v, 0.0) + float(st["ms"][k])
            per_var_b[v] = per_var_b.get(v, 0.0) + bts[k]
            per_var_n[v] = per_var_n.get(v, 0) + 1
    st0 = all_stats[0]
    for k in range(st0["num_levels"]):
        log(f"[bench] level {k}: {B.VARIANT_NAMES[int(st0['variant'][k])]:>16} nF={st0['frontier'][k]} "
            f"eF={st0['frontier_edges'][k]} nU={st0['unvisited'][k]} scan={st0['scanned'][k]} "
            f"next={st0['next'][k]} ms={st0['ms'][k]:.4f}")
    dev_ms = sum(st["elapsed_ms"] for st in all_stats) / len(all_stats)
    per_variant_gbs = {B.VARIANT_NAMES[v]: round(per_var_b[v] / (per_var_t[v] * 1e-3) / 1e9, 1)
                       for v in per_var_t if per_var_t[v] > 0}
    if args.device_loop:
        # one persistent kernel per search: price the whole search per launch
        call_ms = [e0.elapsed_time(e1) for e0, e1 in call_events]
        bytes_per = [sum(bytemodel.level_bytes(st, g.n)) + bytemodel.reset_bytes(g.n) for st in all_stats]
        avg_ms = sum(call_ms) / len(call_ms)
        avg_b = sum(bytes_per) / len(bytes_per)
        achieved = avg_b / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_bfs_persistent (whole search)", "launches": len(call_ms),
                "avg_launch_us": round(avg_ms * 1e3, 2), "bytes_per_launch": round(avg_b),
                "per_level_variant_gbs": per_variant_gbs}
    else:
        dom = max(per_var_t, key=per_var_t.get)
        achieved = per_var_b[dom] / (per_var_t[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": B.VARIANT_NAMES[dom], "launches": per_var_n[dom],
                "avg_launch_us": round(per_var_t[dom] * 1e3 / per_var_n[dom], 2),
                "bytes_per_launch": round(per_var_b[dom] / per_var_n[dom]),
                "time_share": round(per_var_t[dom] / sum(per_var_t.values()), 3),
                "per_variant_gbs": per_variant_gbs}

    extra = {"bfs_device_ms_mean": round(dev_ms, 4),
             "levels_mean": round(float(np.mean([st["num_levels"] for st in all_stats])), 2)}
    if not args.no_sweep:
        sweep = {}
        sub = sources[: args.sweep_sources]
        for v in range(B.NUM_VARIANTS):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sts = one_pass(v, sub, timing=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            sweep[B.VARIANT_NAMES[v]] = round(sum(s["component_edges"] for s in sts) / 2 / dt / 1e9, 3)
        for m, var in (("heuristic", B.AUTO_HEURISTIC),):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sts = one_pass(var, sub, timing=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            sweep[m] = round(sum(s["component_edges"] for s in sts) / 2 / dt / 1e9, 3)
        extra["fixed_and_heuristic_gteps"] = sweep
        extra["sweep_sources"] = len(sub)
        log(f"[bench] sweep {sweep}")
    try:
        t1 = time.perf_counter()
        lvm, stm = B.bfs_multi(dg, sources)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lvm, stm = B.bfs_multi(dg, sources)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        extra["msbfs_64lane_gteps"] = round(stm["component_edges"] / 2 / dt / 1e9, 3)
        del lvm
    except B.BfsError as e:
        extra["msbfs_64lane_gteps"] = None
        log(f"[bench] bfs_multi unavailable: {e}")

    out = {"metric": METRIC, "value": round(gteps, 4), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"{args.workload}-{len(sources)}src", "graph": g.name, "n": g.n, "nnz": g.nnz,
                      "sources": len(sources), "mode": mode, "output": "depths",
                      "level_loop": "device" if args.device_loop else "host"},
           "roofline": roof}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, list(sources), args.cpu_seconds)
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
