"""Trains the per-level variant selector on the GPU.

    python -m paper_2607_17106_amd.train_selector [--out DIR] [--quick]

1. Training states: for each training graph (R-MAT scales 16-22, lattices
   1024^2-4096^2 with deletions and shortcuts) and 16 sources, one search in
   heuristic mode gives exact depths and the per-level counts; level k's state
   is F_k = {depth = k}, P_k = {depth <= k}.
2. Labels: bfs_step_time restores each sampled level's exact state and times
   one step of each of the 4 class variants (median of `reps`).  Every variant
   emits both frontier formats, so switching between levels costs nothing and
   the label of a level is simply its fastest variant (ties to the lowest
   class index).
3. Features: bfs_level_features on the same counts -- the code the device
   selector runs.
4. Training: the library's own kernels (bfs_mlp_loss_grad, bfs_mlp_adam) on
   standardised features; weights are saved with the normalisation, the
   training feature range and the confidence threshold.
5. Evaluation on a held-out R-MAT 22 (graph seed 4922, 64 sources, seed
   4923): summed step time of the learned choice versus the direction
   heuristic, the best single fixed variant and the per-level best (oracle
   schedule), plus end-to-end GTEPS of the learned and heuristic modes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

import graphgen as gg

from . import _lib as L
from . import api, selector

CLASSES = [L.PUSH_Q_BLOCK, L.PUSH_Q_THREAD, L.PUSH_B_NOATOMIC, L.PULL_B]
TRAIN_GRAPHS = [("rmat", s, 4000 + s) for s in range(16, 23)] + \
               [("lattice", 1024, 4110), ("lattice", 2048, 4120), ("lattice", 4096, 4130)]
EVAL_GRAPH = ("rmat", 22, 4922)
EVAL_SOURCES = (64, 4923)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(kind, size, seed):
    return gg.rmat(size, seed=seed) if kind == "rmat" else gg.lattice(size, seed=seed)


def collect(g, sources, reps: int, max_levels_per_source: int):
    """(features [m,12], times [m,4], heuristic variant [m], meta) for the
    sampled levels of searches from `sources`."""
    dg = api.DeviceGraph.from_graph(g)
    depths = torch.empty(g.n, dtype=torch.int32, device="cuda")
    scratch = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ws = torch.empty(api.workspace_size(g.n), dtype=torch.uint8, device="cuda")
    X, T, H, meta = [], [], [], []
    for s in sources:
        _, st = api.bfs_levels(dg, int(s), variant=L.AUTO_HEURISTIC, level_stats=True, levels=depths,
                               workspace=ws)
        F = api.level_features(st, g.n, g.nnz)
        nl = int(st["num_levels"])
        ks = np.unique(np.linspace(0, nl - 1, min(nl, max_levels_per_source)).round().astype(int))
        for k in ks:
            t = [api.step_time(dg, depths, int(k), v, reps=reps, scratch=scratch, workspace=ws) for v in CLASSES]
            X.append(F[k])
            T.append(t)
            H.append(int(st["variant"][k]))
            meta.append((g.name, int(s), int(k)))
    return np.array(X, np.float32), np.array(T, np.float64), np.array(H), meta


def init_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = np.zeros(L.MLP_NPARAM, np.float32)
    for off, fan_in, nout in ((0, 12, 64), (832, 64, 64), (4992, 64, 4)):
        lim = np.sqrt(6.0 / fan_in)
        p[off:off + nout * fan_in] = rng.uniform(-lim, lim, nout * fan_in)
    return p


def train(X, y, steps: int, lr: float, seed: int, batch: int = 512):
    mean = X.mean(0)
    std = X.std(0)
    std = np.where(std > 1e-6, std, 1.0).astype(np.float32)
    Xn = ((X - mean) / std).astype(np.float32)
    p = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    dx = torch.from_numpy(Xn).cuda()
    dy = torch.from_numpy(y.astype(np.int32)).cuda()
    rng = np.random.default_rng(seed)
    losses = []
    for step in range(1, steps + 1):
        if len(y) > batch:
            idx = torch.from_numpy(rng.choice(len(y), batch, replace=False)).cuda()
            xb, yb = dx[idx].contiguous(), dy[idx].contiguous()
        else:
            xb, yb = dx, dy
        g, loss = api.mlp_loss_grad(p, xb, yb)
        api.mlp_adam(p, g, m, v, step, lr * (0.1 ** (step / steps)))
        if step % 100 == 0 or step == 1:
            losses.append((step, float(loss.item())))
    cls, conf = api.mlp_predict(p, dx)
    acc = float((cls.cpu().numpy() == y).mean())
    return p.cpu().numpy(), mean.astype(np.float32), std, losses, acc


def choose(params, mean, std, fmin, fmax, min_conf, X, H):
    """The selector's choice per row (host replica used for evaluation only:
    the device selector makes the same choice from the same numbers)."""
    Xn = ((X - mean) / std).astype(np.float32)
    cls, conf = api.mlp_predict(torch.from_numpy(params).cuda(), torch.from_numpy(Xn).cuda())
    cls, conf = cls.cpu().numpy(), conf.cpu().numpy()
    oor = ((X < fmin) | (X > fmax)).any(axis=1)
    fb = oor | ~(conf >= min_conf)
    pick = np.array(CLASSES)[cls]
    return np.where(fb, H, pick), fb


def schedule_cost(T, chosen):
    idx = {v: i for i, v in enumerate(CLASSES)}
    return float(sum(T[r, idx[int(c)]] for r, c in enumerate(chosen)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.dirname(os.path.abspath(__file__)))
    ap.add_argument("--sources", type=int, default=16)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--levels-per-source", type=int, default=48)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--min-conf", type=float, default=0.4)
    ap.add_argument("--quick", action="store_true", help="small graphs only (smoke run)")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    torch.cuda.set_device(0)
    graphs = TRAIN_GRAPHS if not args.quick else [("rmat", 14, 4014), ("lattice", 256, 4100)]
    Xs, Ts, Hs, metas = [], [], [], []
    t0 = time.time()
    for kind, size, seed in graphs:
        g = make_graph(kind, size, seed)
        srcs = gg.pick_sources(g, args.sources, seed + 1)
        X, T, H, meta = collect(g, srcs, args.reps, args.levels_per_source)
        Xs.append(X); Ts.append(T); Hs.append(H); metas += meta
        log(f"[train] {g.name}: {len(X)} levels ({time.time() - t0:.0f} s)")
    X, T, H = np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Hs)
    y = np.argmin(T, axis=1)
    log(f"[train] {len(y)} samples, label histogram {np.bincount(y, minlength=4).tolist()}")
    params, mean, std, losses, acc = train(X, y, args.steps, args.lr, seed=1)
    span = X.max(0) - X.min(0)
    fmin = (X.min(0) - 0.05 * span - 1e-3).astype(np.float32)
    fmax = (X.max(0) + 0.05 * span + 1e-3).astype(np.float32)
    log(f"[train] loss {losses[0][1]:.3f} -> {losses[-1][1]:.3f}, train accuracy {acc:.3f}")
    out_w = os.path.join(args.out, "selector_weights.npz")
    train_ch, _ = choose(params, mean, std, fmin, fmax, args.min_conf, X, H)
    meta = {"classes": [L.VARIANT_NAMES[c] for c in CLASSES], "samples": int(len(y)),
            "train_accuracy": acc, "losses": losses, "graphs": [f"{k}{s}:{sd}" for k, s, sd in graphs]}
    selector.save(out_w, params, mean, std, fmin, fmax, args.min_conf, CLASSES, meta)

    # held-out evaluation
    kind, size, seed = EVAL_GRAPH if not args.quick else ("rmat", 15, 4915)
    g = make_graph(kind, size, seed)
    srcs = gg.pick_sources(g, EVAL_SOURCES[0] if not args.quick else 8, EVAL_SOURCES[1])
    Xe, Te, He, _ = collect(g, srcs, args.reps, 10 ** 6)
    chosen, fb = choose(params, mean, std, fmin, fmax, args.min_conf, Xe, He)
    best = float(Te.min(axis=1).sum())
    report = {
        "eval_graph": g.name, "eval_seed": seed, "eval_sources": int(len(srcs)), "eval_levels": int(len(Xe)),
        "sum_ms": {"oracle_best_schedule": best, "learned": schedule_cost(Te, chosen),
                   "heuristic": schedule_cost(Te, He),
                   **{f"fixed_{L.VARIANT_NAMES[v]}": float(Te[:, i].sum()) for i, v in enumerate(CLASSES)}},
        "learned_fallback_levels": int(fb.sum()),
        "train": {"samples": int(len(y)), "accuracy": acc, "label_hist": np.bincount(y, minlength=4).tolist(),
                  "train_sum_ms_learned": schedule_cost(T, train_ch), "train_sum_ms_heuristic": schedule_cost(T, H),
                  "train_sum_ms_best": float(T.min(axis=1).sum())},
    }
    # end-to-end on the same sources
    selector.load(out_w)
    dg = api.DeviceGraph.from_graph(g)
    ws = torch.empty(api.workspace_size(g.n), dtype=torch.uint8, device="cuda")
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for mode in (L.AUTO_HEURISTIC, L.AUTO_LEARNED):
        for _ in range(2):  # warm-up pass, then the timed pass
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            edges = 0
            for s in srcs:
                _, st = api.bfs_levels(dg, int(s), variant=mode, workspace=ws, levels=lv)
                edges += st["component_edges"] // 2
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
        report.setdefault("end_to_end_gteps", {})[L.VARIANT_NAMES[mode]] = edges / dt / 1e9
    api.selector_clear()
    with open(os.path.join(args.out, "selector_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps(report))


if __name__ == "__main__":
    main()
