"""Python face of the C ABI: same entry-point names, torch tensors in and out.

Only marshalling happens here: tensors become device pointers, the current
torch stream becomes the hipStream_t, and per-level statistics come back as
numpy arrays.
"""
from __future__ import annotations

import ctypes
import threading
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_i32(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.int32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)


class DeviceGraph:
    """int32 CSR (and CSC) resident on the GPU.  For a symmetric graph the CSC
    arrays alias the CSR ones."""

    def __init__(self, n: int, row_ptr, col_idx, csc_ptr=None, csc_idx=None, symmetric=False,
                 device="cuda"):
        self.n = int(n)
        self.row_ptr = _dev_i32(row_ptr, device)
        self.col_idx = _dev_i32(col_idx, device)
        self.nnz = int(self.col_idx.numel())
        self.symmetric = symmetric
        if symmetric:
            self.csc_ptr, self.csc_idx = self.row_ptr, self.col_idx
        elif csc_ptr is not None:
            self.csc_ptr, self.csc_idx = _dev_i32(csc_ptr, device), _dev_i32(csc_idx, device)
        else:
            self.csc_ptr = self.csc_idx = None
        self._c = L.BfsGraph(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                             self.csc_ptr.data_ptr() if self.csc_ptr is not None else None,
                             self.csc_idx.data_ptr() if self.csc_idx is not None else None)

    @classmethod
    def from_graph(cls, g, device="cuda", with_csc=True):
        """From a graphgen.Graph (host numpy arrays)."""
        if with_csc and not g.symmetric:
            g.with_csc()
            return cls(g.n, g.row_ptr, g.col_idx, g.csc_ptr, g.csc_idx, False, device)
        return cls(g.n, g.row_ptr, g.col_idx, symmetric=g.symmetric and with_csc, device=device)

    @property
    def c(self):
        return ctypes.byref(self._c)

    def graph_sums(self, stream=None):
        """The selector's graph-wide feature sums (bfs_graph_sums), computed on
        first use and kept with the graph."""
        if getattr(self, "_gsums", None) is None:
            ld, ld2 = ctypes.c_int64(0), ctypes.c_int64(0)
            L.check(L.load().bfs_graph_sums(self.c, ctypes.byref(ld), ctypes.byref(ld2), _stream(stream)),
                    "bfs_graph_sums")
            self._gsums = (int(ld.value), int(ld2.value))
        return self._gsums


def _reorder(fn_name, g: DeviceGraph, stream):
    dev = g.row_ptr.device
    i32 = dict(dtype=torch.int32, device=dev)
    rp, ci = torch.empty(g.n + 1, **i32), torch.empty(max(g.nnz, 1), **i32)
    own_csc = g.csc_ptr is not None and not g.symmetric
    cp = torch.empty(g.n + 1, **i32) if own_csc else None
    cx = torch.empty(max(g.nnz, 1), **i32) if own_csc else None
    new_of_old, old_of_new = torch.empty(g.n, **i32), torch.empty(g.n, **i32)
    rc = getattr(L.load(), fn_name)(g.c, _ptr(rp), _ptr(ci), _ptr(cp), _ptr(cx), _ptr(new_of_old),
                                    _ptr(old_of_new), _stream(stream))
    L.check(rc, fn_name)
    ci = ci[:g.nnz]
    if own_csc:
        out = DeviceGraph(g.n, rp, ci, cp, cx[:g.nnz], symmetric=False, device=dev)
    else:
        out = DeviceGraph(g.n, rp, ci, symmetric=g.symmetric, device=dev)
    return out, new_of_old, old_of_new


def reorder_degree(g: DeviceGraph, stream=None):
    """bfs_reorder_degree: the graph renumbered by decreasing out-degree.
    Returns (renumbered DeviceGraph, new_of_old, old_of_new), the maps as
    device int32 tensors; pass new_of_old as bfs_multi's vertex_map.  The
    returned graph is marked hub_order (bfs_multi then sets F_HUB_ORDER)."""
    out, n2o, o2n = _reorder("bfs_reorder_degree", g, stream)
    out.hub_order = True
    return out, n2o, o2n


def reorder_rcm(g: DeviceGraph, stream=None):
    """bfs_reorder_rcm: the graph renumbered by reverse Cuthill-McKee (same
    return values as reorder_degree)."""
    return _reorder("bfs_reorder_rcm", g, stream)


def workspace_size(n: int, lanes: int = 1) -> int:
    b = ctypes.c_size_t(0)
    L.check(L.load().bfs_workspace_size(n, lanes, ctypes.byref(b)), "bfs_workspace_size")
    return int(b.value)


class _StatsBuf:
    """Host arrays the library fills with per-level statistics.  One buffer
    per thread and capacity is kept and reused (get()): building the ctypes
    view costs far more than a short search's host work."""
    _local = threading.local()

    @classmethod
    def get(cls, cap: int) -> "_StatsBuf":
        cache = getattr(cls._local, "bufs", None)
        if cache is None:
            cache = cls._local.bufs = {}
        buf = cache.get(cap)
        if buf is None:
            buf = cache[cap] = cls(cap)
        # a call fills only the fields its path knows: clear what the last
        # call may have written (every entry, if it never reached as_dict)
        s = buf.s
        s.num_levels = s.fell_back = s.host_syncs = 0
        s.reached = s.component_edges = s.graph_ld = s.graph_ld2 = 0
        s.elapsed_ms = 0.0
        for a in buf._arrays:
            a[:buf._dirty] = 0
        buf._dirty = cap
        return buf

    def __init__(self, cap: int):
        self.cap = cap
        self.variant = np.zeros(cap, np.int32)
        self.frontier = np.zeros(cap, np.int64)
        self.frontier_edges = np.zeros(cap, np.int64)
        self.unvisited = np.zeros(cap, np.int64)
        self.unvisited_edges = np.zeros(cap, np.int64)
        self.fallback = np.zeros(cap, np.int32)
        self.fld = np.zeros(cap, np.int64)
        self.fld2 = np.zeros(cap, np.int64)
        self.scanned = np.zeros(cap, np.int64)
        self.nxt = np.zeros(cap, np.int64)
        self.ms = np.zeros(cap, np.float32)
        self.ms_main = np.zeros(cap, np.float32)
        self.scan_aux = np.zeros(cap, np.int64)
        self.hits_aux = np.zeros(cap, np.int64)
        self.scan_push = np.zeros(cap, np.int64)
        self.push_src = np.zeros(cap, np.int64)
        self._arrays = (self.variant, self.frontier, self.frontier_edges, self.unvisited, self.unvisited_edges,
                        self.fallback, self.fld, self.fld2, self.scanned, self.nxt, self.ms, self.ms_main,
                        self.scan_aux, self.hits_aux, self.scan_push, self.push_src)
        self._dirty = 0
        P32, P64 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        self.s = L.BfsStats()
        self.s.level_capacity = cap
        self.s.level_variant = self.variant.ctypes.data_as(P32)
        self.s.level_frontier = self.frontier.ctypes.data_as(P64)
        self.s.level_frontier_edges = self.frontier_edges.ctypes.data_as(P64)
        self.s.level_unvisited = self.unvisited.ctypes.data_as(P64)
        self.s.level_unvisited_edges = self.unvisited_edges.ctypes.data_as(P64)
        self.s.level_fallback = self.fallback.ctypes.data_as(P32)
        self.s.level_frontier_ld = self.fld.ctypes.data_as(P64)
        self.s.level_frontier_ld2 = self.fld2.ctypes.data_as(P64)
        self.s.level_scanned = self.scanned.ctypes.data_as(P64)
        self.s.level_next = self.nxt.ctypes.data_as(P64)
        self.s.level_ms = self.ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self.s.level_ms_main = self.ms_main.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self.s.level_scanned_aux = self.scan_aux.ctypes.data_as(P64)
        self.s.level_hits_aux = self.hits_aux.ctypes.data_as(P64)
        self.s.level_scanned_push = self.scan_push.ctypes.data_as(P64)
        self.s.level_push_sources = self.push_src.ctypes.data_as(P64)

    def as_dict(self, per_level: bool):
        s = self.s
        d = dict(num_levels=s.num_levels, fell_back=s.fell_back, reached=s.reached,
                 component_edges=s.component_edges, elapsed_ms=s.elapsed_ms, host_syncs=s.host_syncs,
                 graph_ld=s.graph_ld, graph_ld2=s.graph_ld2)
        self._dirty = min(max(s.num_levels, 0), self.cap)
        if per_level:
            k = self._dirty
            d.update(variant=self.variant[:k].copy(), frontier=self.frontier[:k].copy(),
                     frontier_edges=self.frontier_edges[:k].copy(), unvisited=self.unvisited[:k].copy(),
                     unvisited_edges=self.unvisited_edges[:k].copy(), fallback=self.fallback[:k].copy(),
                     frontier_ld=self.fld[:k].copy(), frontier_ld2=self.fld2[:k].copy(),
                     scanned=self.scanned[:k].copy(), next=self.nxt[:k].copy(), ms=self.ms[:k].copy(),
                     ms_main=self.ms_main[:k].copy(), scanned_aux=self.scan_aux[:k].copy(),
                     hits_aux=self.hits_aux[:k].copy(), scanned_push=self.scan_push[:k].copy(),
                     push_sources=self.push_src[:k].copy())
        return d


def _options(variant, flags, schedule, workspace, max_levels, heuristic_push):
    opt = L.BfsOptions()
    opt.variant = int(variant)
    opt.flags = int(flags)
    opt.max_levels = int(max_levels)
    opt.heuristic_push = -1 if heuristic_push is None else int(heuristic_push)
    opt.heuristic_pull = -1
    keep = []
    if schedule is not None:
        arr = np.ascontiguousarray(schedule, dtype=np.int32)
        keep.append(arr)
        opt.schedule_host = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        opt.schedule_len = int(arr.size)
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    return opt, keep


def _check_vmap(g, vertex_map):
    if vertex_map.dtype != torch.int32 or vertex_map.numel() != g.n or not vertex_map.is_contiguous():
        raise ValueError("vertex_map must be a contiguous int32 tensor of n entries")
    return vertex_map.data_ptr()


def _run_single(fn_name, g: DeviceGraph, source, want_parents, variant, flags, schedule, level_stats,
                workspace, levels, parents, max_levels, heuristic_push, stream, stats_capacity, vertex_map=None):
    lib = L.load()
    dev = g.row_ptr.device
    if levels is None:
        levels = torch.empty(g.n, dtype=torch.int32, device=dev)
    if want_parents and parents is None:
        parents = torch.empty(g.n, dtype=torch.int32, device=dev)
    if flags & L.F_LEVEL_TIMING:
        level_stats = True
    if level_stats:
        flags |= L.F_LEVEL_STATS
    sb = _StatsBuf.get(stats_capacity if level_stats else 0)
    opt, keep = _options(variant, flags, schedule, workspace, max_levels, heuristic_push)
    if variant == L.AUTO_LEARNED or level_stats:
        opt.graph_ld, opt.graph_ld2 = g.graph_sums(stream)
        opt.flags |= L.F_GRAPH_SUMS
    if vertex_map is not None:
        opt.vertex_map = _check_vmap(g, vertex_map)
    if want_parents:
        rc = lib.bfs_parents(g.c, int(source), _ptr(levels), _ptr(parents), ctypes.byref(opt),
                             ctypes.byref(sb.s), _stream(stream))
    else:
        rc = lib.bfs_levels(g.c, int(source), _ptr(levels), ctypes.byref(opt), ctypes.byref(sb.s),
                            _stream(stream))
    L.check(rc, fn_name)
    del keep
    return levels, parents, sb.as_dict(level_stats)


def bfs_levels(g: DeviceGraph, source: int, variant: int = L.AUTO_HEURISTIC, flags: int = 0,
               schedule: Optional[Sequence[int]] = None, level_stats: bool = False, workspace=None,
               levels=None, max_levels: int = 0, heuristic_push=None, stream=None,
               stats_capacity: int = 1 << 16, vertex_map=None):
    """Depths from `source`; returns (levels int32 tensor, stats dict).
    vertex_map: the new_of_old of a renumbering when g is the renumbered graph
    (source and depths then use the original ids)."""
    lv, _, st = _run_single("bfs_levels", g, source, False, variant, flags, schedule, level_stats, workspace,
                            levels, None, max_levels, heuristic_push, stream, stats_capacity, vertex_map)
    return lv, st


def bfs_parents(g: DeviceGraph, source: int, variant: int = L.AUTO_HEURISTIC, flags: int = 0,
                schedule: Optional[Sequence[int]] = None, level_stats: bool = False, workspace=None,
                levels=None, parents=None, max_levels: int = 0, heuristic_push=None, stream=None,
                stats_capacity: int = 1 << 16, vertex_map=None):
    """Depths and a valid BFS parent per vertex; returns (levels, parents, stats).
    vertex_map as for bfs_levels (parents are then original ids too)."""
    return _run_single("bfs_parents", g, source, True, variant, flags, schedule, level_stats, workspace,
                       levels, parents, max_levels, heuristic_push, stream, stats_capacity, vertex_map)


def bfs_levels_noalloc(g: DeviceGraph, source: int, variant: int = L.AUTO_HEURISTIC, flags: int = 0,
                       schedule: Optional[Sequence[int]] = None, levels=None, max_levels: int = 0,
                       heuristic_push=None, stream=None, vertex_map=None):
    """bfs_levels_noalloc: depths from `source` with the library's static
    scratch (no workspace, nothing allocated by the call); returns (levels,
    stats dict without per-level arrays)."""
    if levels is None:
        levels = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
    sb = _StatsBuf.get(0)
    opt, keep = _options(variant, flags, schedule, None, max_levels, heuristic_push)
    if vertex_map is not None:
        opt.vertex_map = _check_vmap(g, vertex_map)
    rc = L.load().bfs_levels_noalloc(g.c, int(source), _ptr(levels), ctypes.byref(opt), ctypes.byref(sb.s),
                                     _stream(stream))
    L.check(rc, "bfs_levels_noalloc")
    del keep
    return levels, sb.as_dict(False)


@dataclass
class MultiConfig:
    """bfs_multi_config: the tunable choices of bfs_multi's level steps (0 = the library default)."""
    wide_ratio: int = 0
    split_vpt: int = 0
    cap0: int = 0
    tile_alpha: int = 0
    alpha: int = 0
    split_lout: int = 0
    wide_vpt: int = 0
    narrow_vpt: int = 0

    def c(self):
        return L.BfsMultiConfig(self.wide_ratio, self.split_vpt, self.cap0, self.tile_alpha, self.alpha,
                                self.split_lout, self.wide_vpt, self.narrow_vpt)


def _multi_options(g, variant, flags, workspace, vertex_map, hub_split, config):
    if getattr(g, "hub_order", False):
        flags |= L.F_HUB_ORDER
    opt, keep = _options(variant, flags, None, workspace, 0, None)
    if vertex_map is not None:
        opt.vertex_map = _check_vmap(g, vertex_map)
    opt.hub_split = int(hub_split)
    if config is not None:
        cc = config.c()
        keep.append(cc)
        opt.multi_config = ctypes.pointer(cc)
    return opt, keep


def bfs_multi(g: DeviceGraph, sources, variant: int = L.AUTO_HEURISTIC, flags: int = 0, workspace=None,
              levels=None, stream=None, level_stats: bool = False, stats_capacity: int = 1 << 14,
              vertex_map=None, hub_split: int = 0, config: MultiConfig = None):
    """Depths [k][n] from k sources in 64-lane bit-packed groups.  vertex_map:
    the new_of_old of reorder_degree when g is the renumbered graph (sources
    and depth columns then use the original ids).  hub_split: the split id of
    split bottom-up levels (0 automatic, > 0 that id on every bottom-up level,
    < 0 never; bfs_options.hub_split).  config: a MultiConfig, or None for the
    one bfs_multi_autotune stored for this graph (else the defaults)."""
    lib = L.load()
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.size)
    if levels is None:
        levels = torch.empty((max(k, 1), g.n), dtype=torch.int32, device=g.row_ptr.device)
    if flags & (L.F_LEVEL_TIMING | L.F_MAIN_TIMING):
        level_stats = True
    if level_stats:
        flags |= L.F_LEVEL_STATS
    sb = _StatsBuf.get(stats_capacity if level_stats else 0)
    opt, keep = _multi_options(g, variant, flags, workspace, vertex_map, hub_split, config)
    rc = lib.bfs_multi(g.c, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), k, _ptr(levels),
                       ctypes.byref(opt), ctypes.byref(sb.s), _stream(stream))
    L.check(rc, "bfs_multi")
    del keep
    return levels[:k], sb.as_dict(level_stats)


def bfs_multi_autotune(g: DeviceGraph, sources, variant: int = L.AUTO_HEURISTIC, flags: int = 0, workspace=None,
                       levels=None, stream=None, vertex_map=None, hub_split: int = 0, config: MultiConfig = None):
    """bfs_multi_autotune: the fastest MultiConfig for this graph and source
    set (stored by the library for later bfs_multi calls on the graph) and
    its device time in ms."""
    lib = L.load()
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.size)
    if levels is None:
        levels = torch.empty((max(k, 1), g.n), dtype=torch.int32, device=g.row_ptr.device)
    opt, keep = _multi_options(g, variant, flags, workspace, vertex_map, hub_split, config)
    best = L.BfsMultiConfig()
    ms = ctypes.c_float(0.0)
    rc = lib.bfs_multi_autotune(g.c, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), k, _ptr(levels),
                                ctypes.byref(opt), ctypes.byref(best), ctypes.byref(ms), _stream(stream))
    L.check(rc, "bfs_multi_autotune")
    del keep
    return MultiConfig(best.wide_ratio, best.split_vpt, best.cap0, best.tile_alpha, best.alpha,
                       best.split_lout, best.wide_vpt, best.narrow_vpt), float(ms.value)


@dataclass
class BatchConfig:
    block_threads: int = 1024
    small_vertices: int = 1 << 20
    blocks_per_cu: int = 2
    team_vertices: int = 131072
    max_team: int = 8

    def c(self, workspace=None):
        c = L.BfsBatchConfig(self.block_threads, self.small_vertices, self.blocks_per_cu,
                             self.team_vertices, self.max_team, None, 0)
        if workspace is not None:
            c.workspace = workspace.data_ptr()
            c.workspace_bytes = workspace.numel() * workspace.element_size()
        return c

    @classmethod
    def from_c(cls, c):
        return cls(c.block_threads, c.small_vertices, c.blocks_per_cu, c.team_vertices, c.max_team)


class DeviceBatch:
    """A graphgen.GraphBatch resident on the GPU."""

    def __init__(self, b, device="cuda"):
        self.num = b.num
        self.total_n = b.total_n
        self.total_nnz = b.total_nnz
        self.v_off = np.ascontiguousarray(b.v_off, dtype=np.int64)
        self.e_off = np.ascontiguousarray(b.e_off, dtype=np.int64)
        self.row_ptr = _dev_i32(b.row_ptr, device)
        self.col_idx = _dev_i32(b.col_idx, device)
        self.sources = np.ascontiguousarray(b.sources, dtype=np.int32)
        P64 = ctypes.POINTER(ctypes.c_int64)
        self.symmetric = all(g.symmetric for g in b.graphs)
        self._c = L.BfsGraphBatch(self.num, self.total_n, self.total_nnz, self.v_off.ctypes.data_as(P64),
                                  self.e_off.ctypes.data_as(P64), self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                                  1 if self.symmetric else 0)

    @property
    def c(self):
        return ctypes.byref(self._c)


def batch_workspace_size(b: DeviceBatch, config: Optional[BatchConfig] = None, sources=None) -> int:
    src = np.ascontiguousarray(b.sources if sources is None else sources, dtype=np.int32)
    cfg = config.c() if config is not None else None
    nb = ctypes.c_size_t(0)
    L.check(L.load().bfs_batch_workspace_size(b.c, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(nb)),
            "bfs_batch_workspace_size")
    return int(nb.value)


def bfs_batch(b: DeviceBatch, sources=None, config: Optional[BatchConfig] = None, levels=None, stream=None,
              workspace=None):
    """With a config, the scratch is a caller tensor (`workspace`, else one
    allocated here of bfs_batch_workspace_size bytes); without one the library
    uses the default or autotuned config and a buffer it keeps."""
    lib = L.load()
    src = np.ascontiguousarray(b.sources if sources is None else sources, dtype=np.int32)
    if levels is None:
        levels = torch.empty(b.total_n, dtype=torch.int32, device=b.row_ptr.device)
    sb = _StatsBuf.get(0)
    cfg = None
    if config is not None:
        if workspace is None:
            workspace = torch.empty(batch_workspace_size(b, config, src), dtype=torch.uint8,
                                    device=b.row_ptr.device)
        cfg = config.c(workspace)
    rc = lib.bfs_batch(b.c, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(levels),
                       ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(sb.s), _stream(stream))
    L.check(rc, "bfs_batch")
    return levels, sb.as_dict(False)


def bfs_batch_autotune(b: DeviceBatch, sources=None, levels=None, stream=None, workspace=None):
    lib = L.load()
    src = np.ascontiguousarray(b.sources if sources is None else sources, dtype=np.int32)
    if levels is None:
        levels = torch.empty(b.total_n, dtype=torch.int32, device=b.row_ptr.device)
    best = L.BfsBatchConfig()
    if workspace is not None:
        best.workspace = workspace.data_ptr()
        best.workspace_bytes = workspace.numel() * workspace.element_size()
    ms = ctypes.c_float(0)
    rc = lib.bfs_batch_autotune(b.c, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(levels),
                                ctypes.byref(best), ctypes.byref(ms), _stream(stream))
    L.check(rc, "bfs_batch_autotune")
    return BatchConfig.from_c(best), float(ms.value)


# ------------------------------------------------------------------ selector

def _f32p(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def selector_set(params, mean, std, fmin, fmax, min_confidence: float, class_variants):
    keep = [_f32p(x) for x in (params, mean, std, fmin, fmax)]
    cv = np.ascontiguousarray(class_variants, dtype=np.int32)
    rc = L.load().bfs_selector_set(*[k[1] for k in keep], float(min_confidence),
                                   cv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    L.check(rc, "bfs_selector_set")


def selector_clear():
    L.check(L.load().bfs_selector_clear(), "bfs_selector_clear")


def selector_loaded() -> bool:
    return bool(L.load().bfs_selector_loaded())


def mlp_forward(params: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
    B = x.shape[0]
    out = torch.empty((B, L.MLP_NCLASS), dtype=torch.float32, device=x.device)
    L.check(L.load().bfs_mlp_forward(_ptr(params), _ptr(x), B, _ptr(out), _stream(stream)), "bfs_mlp_forward")
    return out


def mlp_predict(params: torch.Tensor, x: torch.Tensor, stream=None):
    B = x.shape[0]
    cls = torch.empty(B, dtype=torch.int32, device=x.device)
    conf = torch.empty(B, dtype=torch.float32, device=x.device)
    L.check(L.load().bfs_mlp_predict(_ptr(params), _ptr(x), B, _ptr(cls), _ptr(conf), _stream(stream)),
            "bfs_mlp_predict")
    return cls, conf


def mlp_loss_grad(params: torch.Tensor, x: torch.Tensor, labels: torch.Tensor, grad=None, loss=None, stream=None):
    B = x.shape[0]
    if grad is None:
        grad = torch.empty(L.MLP_NPARAM, dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    L.check(L.load().bfs_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(labels), B, _ptr(grad), _ptr(loss),
                                       _stream(stream)), "bfs_mlp_loss_grad")
    return grad, loss


def mlp_adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    L.check(L.load().bfs_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                                  float(beta2), float(eps), _stream(stream)), "bfs_mlp_adam")


def level_features(stats: dict, n: int, nnz: int) -> np.ndarray:
    """Raw selector features of each level of a finished search (stats from a
    bfs_levels/bfs_parents call with level_stats=True)."""
    k = int(stats["num_levels"])
    sb = _StatsBuf(k)
    sb.s.num_levels = k
    sb.s.graph_ld = int(stats["graph_ld"])
    sb.s.graph_ld2 = int(stats["graph_ld2"])
    sb.frontier[:] = stats["frontier"]
    sb.frontier_edges[:] = stats["frontier_edges"]
    sb.unvisited[:] = stats["unvisited"]
    sb.unvisited_edges[:] = stats["unvisited_edges"]
    sb.fld[:] = stats["frontier_ld"]
    sb.fld2[:] = stats["frontier_ld2"]
    out = np.zeros((k, L.MLP_NFEAT), dtype=np.float32)
    L.check(L.load().bfs_level_features(ctypes.byref(sb.s), int(n), int(nnz),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "bfs_level_features")
    return out


def step_time(g: DeviceGraph, depths: torch.Tensor, k: int, variant: int, reps: int = 3, scratch=None,
              workspace=None, stream=None) -> float:
    """Median device time (ms) of one step of `variant` from the exact state of level k."""
    if scratch is None:
        scratch = torch.empty(g.n, dtype=torch.int32, device=depths.device)
    opt, keep = _options(0, 0, None, workspace, 0, None)
    ms = ctypes.c_float(0)
    L.check(L.load().bfs_step_time(g.c, _ptr(depths), int(k), int(variant), int(reps), _ptr(scratch),
                                   ctypes.byref(opt), ctypes.byref(ms), _stream(stream)), "bfs_step_time")
    return float(ms.value)
