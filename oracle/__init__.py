"""CPU oracle for the BFS level step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It shares no code with the HIP
library and never imports it; the two meet only through the seeded inputs of
``graphgen``.

Contents
  bfs(...)            plain FIFO-queue BFS (C, bfs_oracle.c): depths, parents
  level_profile(...)  per-level |F|, frontier edges, |U|, unvisited in-edges,
                      bottom-up early-exit scan length
  multi(...), batch(...)  one oracle BFS per source / per instance
  brute               all-pairs unit-weight distances (Floyd-Warshall)
  checks              Graph500-style parent validation and level invariants
  mlp                 fp64 reference of the selector network
  heuristic           replay of the direction-optimising rule
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_liboracle.so")
_SRC = os.path.join(_HERE, "bfs_oracle.c")


def build(force: bool = False) -> str:
    """Compiles the C oracle (plain gcc -O3, single thread, portable ISA)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.oracle_bfs.restype = ctypes.c_int32
        lib.oracle_bfs.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, P, P]
        lib.oracle_level_profile.restype = None
        lib.oracle_level_profile.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int32,
                                             P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def bfs(row_ptr, col_idx, source: int, want_parents: bool = True):
    """Returns (levels, parents or None, num_levels)."""
    row_ptr = _i32(row_ptr)
    col_idx = _i32(col_idx)
    n = row_ptr.shape[0] - 1
    lev = np.empty(n, dtype=np.int32)
    par = np.empty(n, dtype=np.int32) if want_parents else None
    q = np.empty(n, dtype=np.int32)
    nl = _L().oracle_bfs(n, _p(row_ptr), _p(col_idx), int(source), _p(lev),
                         _p(par) if want_parents else None, _p(q))
    if nl < 0:
        raise ValueError("oracle_bfs: bad input (n <= 0 or source out of range)")
    return lev, par, int(nl)


def level_profile(row_ptr, csc_ptr, csc_idx, levels):
    """Dict of int64 arrays nF, eF, nU, eU, eScan indexed by level."""
    levels = _i32(levels)
    nlev = int(levels.max()) + 1 if levels.size and levels.max() >= 0 else 0
    out = {k: np.zeros(max(nlev, 1), dtype=np.int64) for k in ("nF", "eF", "nU", "eU", "eScan")}
    if nlev:
        _L().oracle_level_profile(levels.shape[0], _p(_i32(row_ptr)), _p(_i32(csc_ptr)),
                                  _p(_i32(csc_idx)), _p(levels), nlev, _p(out["nF"]),
                                  _p(out["eF"]), _p(out["nU"]), _p(out["eU"]), _p(out["eScan"]))
    return {k: v[:nlev] for k, v in out.items()}


def host_threads() -> int:
    """Threads for the per-source loops: the host's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def _map(fn, items, threads):
    """fn over items, one oracle search per host thread (the C search runs
    with the interpreter lock released); results in item order."""
    items = list(items)
    threads = host_threads() if threads is None else max(1, int(threads))
    if threads == 1 or len(items) <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(max_workers=min(threads, len(items))) as ex:
        return list(ex.map(fn, items))


def multi(row_ptr, col_idx, sources, threads=None):
    """Levels [k][n] of one oracle BFS per source (the multi-source BFS with
    one lane per source computes exactly these).  The searches are
    independent; up to `threads` run at once."""
    row_ptr = _i32(row_ptr)
    col_idx = _i32(col_idx)
    n = len(row_ptr) - 1
    out = np.empty((len(sources), n), dtype=np.int32)

    def one(i):
        out[i] = bfs(row_ptr, col_idx, int(sources[i]), want_parents=False)[0]

    _map(one, range(len(sources)), threads)
    return out


def batch(batch_graphs, sources, threads=None):
    """Per-instance levels (local ids), concatenated in instance order."""
    pairs = list(zip(batch_graphs, sources))
    parts = _map(lambda gs: bfs(gs[0].row_ptr, gs[0].col_idx, int(gs[1]), want_parents=False)[0], pairs, threads)
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int32)


def edges_in_component(row_ptr, levels) -> int:
    """Sum of out-degrees of reached vertices (CSR entries of the traversed
    component)."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    return int(deg[np.asarray(levels) >= 0].sum())
