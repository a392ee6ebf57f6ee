"""Seeded synthetic graphs for the BFS library and its CPU oracle.

This module is input preparation only and holds none of the breadth-first
search arithmetic.  Both the HIP path (tests, benchmark) and the oracle use
it, so it must never import either of them.

Families (the paper's 36 real graphs are not available; these stand in for its
high-degree-variance Kronecker group and its low-variance road-like group):

* ``rmat``      R-MAT/Kronecker, a,b,c,d = .57,.19,.19,.05, edge factor 16,
                seeded vertex relabel, symmetrised, self-loops and duplicate
                edges removed, rows sorted ascending.
* ``lattice``   side x side 4-neighbour grid, each edge deleted with
                probability 0.10, then round(0.001 * lattice edges) uniform
                random shortcuts, symmetrised and deduplicated.
* ``erdos_renyi`` G(n, m) with m = n * mean_degree / 2 uniform pairs.
* ``directed_random`` small directed graphs (CSC differs from CSR) for tests.

Random numbers are counter based (see gen.c), so every graph depends only on
its parameters and seed.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_libgraphgen.so")
_SRC = os.path.join(_HERE, "gen.c")


def build(force: bool = False) -> str:
    """Compiles gen.c into _libgraphgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gg_rng.restype = u64
        lib.gg_rng.argtypes = [u64, u64, u64]
        lib.gg_rmat_edges.argtypes = [i32, i64, dbl, dbl, dbl, u64, P, P]
        lib.gg_permutation.argtypes = [i64, u64, P]
        lib.gg_apply_perm.argtypes = [i64, P, P]
        lib.gg_lattice_edges.restype = i64
        lib.gg_lattice_edges.argtypes = [i32, dbl, i64, u64, P, P]
        lib.gg_uniform_pairs.argtypes = [i64, i64, u64, u64, P, P]
        lib.gg_build_csr.restype = i64
        lib.gg_build_csr.argtypes = [i64, i64, P, P, i32, i32, i32, P, P]
        lib.gg_transpose.argtypes = [i64, P, P, P, P]
        lib.gg_largest_component.restype = i64
        lib.gg_largest_component.argtypes = [i64, P, P, P]
        lib.gg_pick_sources.restype = i32
        lib.gg_pick_sources.argtypes = [i64, P, P, P, i32, u64, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """A directed graph in int32 CSR; ``csc_*`` is its transpose (the same
    arrays when the graph is symmetric)."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    symmetric: bool
    name: str = ""
    csc_ptr: Optional[np.ndarray] = None
    csc_idx: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def with_csc(self) -> "Graph":
        if self.csc_ptr is None:
            if self.symmetric:
                self.csc_ptr, self.csc_idx = self.row_ptr, self.col_idx
            else:
                self.csc_ptr, self.csc_idx = transpose(self.n, self.row_ptr, self.col_idx)
        return self

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, symmetrize: bool = True,
                   drop_self: bool = True, dedup: bool = True):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    if m and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(1, (2 * m) if symmetrize else m), dtype=np.int32)
    nnz = _L().gg_build_csr(n, m, _p(src), _p(dst), int(symmetrize), int(drop_self), int(dedup),
                            _p(row_ptr), _p(col))
    if nnz < 0:
        raise ValueError("graph does not fit an int32 CSR (nnz >= 2^31)")
    return row_ptr, col[:nnz].copy()


def transpose(n: int, row_ptr: np.ndarray, col_idx: np.ndarray):
    t_ptr = np.empty(n + 1, dtype=np.int32)
    t_col = np.empty(max(1, int(row_ptr[-1])), dtype=np.int32)
    _L().gg_transpose(n, _p(row_ptr), _p(col_idx), _p(t_ptr), _p(t_col))
    return t_ptr, t_col[: int(row_ptr[-1])].copy()


# ---------------------------------------------------------------------------
# on-disk cache (big graphs take seconds to build; the key covers every input)

def _cache_dir() -> Optional[str]:
    d = os.environ.get("BFS_GRAPH_CACHE", "/tmp/bfs_graph_cache")
    if d in ("", "0", "off"):
        return None
    os.makedirs(d, exist_ok=True)
    return d


def _cached(key: str, make):
    d = _cache_dir()
    tag = hashlib.sha1((key + open(_SRC, "rb").read().hex()[:64]).encode()).hexdigest()[:20]
    if d is not None:
        f = os.path.join(d, tag + ".npz")
        if os.path.exists(f):
            with np.load(f, allow_pickle=False) as z:
                return z["row_ptr"], z["col_idx"]
    row_ptr, col = make()
    if d is not None and row_ptr.shape[0] > 100_000:
        tmp = os.path.join(d, tag + ".tmp%d.npz" % os.getpid())
        np.savez(tmp, row_ptr=row_ptr, col_idx=col)
        os.replace(tmp, os.path.join(d, tag + ".npz"))
    return row_ptr, col


# ---------------------------------------------------------------------------
# families

def rmat(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, relabel: bool = True) -> Graph:
    n = 1 << scale
    m = edgefactor * n

    def make():
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        L = _L()
        L.gg_rmat_edges(scale, m, a, b, c, seed, _p(src), _p(dst))
        if relabel:
            perm = np.empty(n, dtype=np.int32)
            L.gg_permutation(n, seed, _p(perm))
            L.gg_apply_perm(m, _p(perm), _p(src))
            L.gg_apply_perm(m, _p(perm), _p(dst))
        return csr_from_edges(n, src, dst, True, True, True)

    row_ptr, col = _cached(f"rmat:{scale}:{edgefactor}:{a}:{b}:{c}:{seed}:{relabel}", make)
    return Graph(n, row_ptr, col, True, name=f"rmat{scale}",
                 meta=dict(kind="rmat", scale=scale, edgefactor=edgefactor, tuples=m, seed=seed))


def lattice_shortcut_count(side: int, shortcut_frac: float = 0.001) -> int:
    return int(round(shortcut_frac * 2 * side * (side - 1)))


def lattice(side: int, p_delete: float = 0.10, shortcut_frac: float = 0.001, seed: int = 1) -> Graph:
    n = side * side
    ne = 2 * side * (side - 1)
    sc = lattice_shortcut_count(side, shortcut_frac)

    def make():
        src = np.empty(ne + sc, dtype=np.int32)
        dst = np.empty(ne + sc, dtype=np.int32)
        w = _L().gg_lattice_edges(side, p_delete, sc, seed, _p(src), _p(dst))
        return csr_from_edges(n, src[:w], dst[:w], True, True, True)

    row_ptr, col = _cached(f"lattice:{side}:{p_delete}:{shortcut_frac}:{seed}", make)
    return Graph(n, row_ptr, col, True, name=f"lattice{side}",
                 meta=dict(kind="lattice", side=side, p_delete=p_delete, shortcuts=sc, seed=seed))


def erdos_renyi(n: int, mean_degree: float = 8.0, seed: int = 1) -> Graph:
    m = int(round(n * mean_degree / 2))

    def make():
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        _L().gg_uniform_pairs(n, m, seed, 5, _p(src), _p(dst))
        return csr_from_edges(n, src, dst, True, True, True)

    row_ptr, col = _cached(f"er:{n}:{mean_degree}:{seed}", make)
    return Graph(n, row_ptr, col, True, name=f"er{n}",
                 meta=dict(kind="er", pairs=m, seed=seed))


def directed_random(n: int, m: int, seed: int = 1, self_loops: bool = False,
                    duplicates: bool = False) -> Graph:
    """Directed graph (CSC != CSR) from m uniform ordered pairs.  With
    ``self_loops``/``duplicates`` those tuples are kept in the CSR."""
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _L().gg_uniform_pairs(n, m, seed, 7, _p(src), _p(dst))
    row_ptr, col = csr_from_edges(n, src, dst, symmetrize=False, drop_self=not self_loops,
                                  dedup=not duplicates)
    return Graph(n, row_ptr, col, False, name=f"dir{n}_{m}").with_csc()


def from_edge_list(n: int, edges, symmetric: bool, name: str = "") -> Graph:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    row_ptr, col = csr_from_edges(n, e[:, 0], e[:, 1], symmetrize=symmetric, drop_self=False,
                                  dedup=False)
    return Graph(n, row_ptr, col, symmetric, name=name).with_csc()


# ---------------------------------------------------------------------------
# sources

def largest_component_mask(g: Graph) -> np.ndarray:
    mask = np.zeros(g.n, dtype=np.uint8)
    _L().gg_largest_component(g.n, _p(g.row_ptr), _p(g.col_idx), _p(mask))
    return mask


def pick_sources(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct vertices drawn uniformly from the largest weakly connected
    component among those with at least two neighbours other than
    themselves (degree > 1, self-loops excluded, as in Graph500 practice)."""
    mask = largest_component_mask(g)
    out = np.empty(max(1, k), dtype=np.int32)
    got = _L().gg_pick_sources(g.n, _p(g.row_ptr), _p(g.col_idx), _p(mask), k, seed, _p(out))
    return out[:got].copy()


# ---------------------------------------------------------------------------
# batches of independent graphs (concatenated CSR with per-instance offsets)

@dataclass
class GraphBatch:
    """B graphs stored back to back.  Instance b owns global vertices
    [v_off[b], v_off[b+1]) and CSR entries [e_off[b], e_off[b+1]).
    ``row_ptr`` has one entry per vertex plus a final one and holds GLOBAL
    entry offsets; ``col_idx`` holds LOCAL vertex ids (0 .. n_b-1)."""
    graphs: List[Graph]
    v_off: np.ndarray
    e_off: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    sources: np.ndarray  # local source id per instance

    @property
    def num(self) -> int:
        return len(self.graphs)

    @property
    def total_n(self) -> int:
        return int(self.v_off[-1])

    @property
    def total_nnz(self) -> int:
        return int(self.e_off[-1])


def concat(graphs: List[Graph], sources) -> GraphBatch:
    B = len(graphs)
    v_off = np.zeros(B + 1, dtype=np.int64)
    e_off = np.zeros(B + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        v_off[i + 1] = v_off[i] + g.n
        e_off[i + 1] = e_off[i] + g.nnz
    if e_off[-1] >= 2 ** 31 or v_off[-1] >= 2 ** 31:
        raise ValueError("batch too large for int32 offsets")
    row_ptr = np.empty(int(v_off[-1]) + 1, dtype=np.int32)
    col = np.empty(max(1, int(e_off[-1])), dtype=np.int32)
    for i, g in enumerate(graphs):
        row_ptr[v_off[i]:v_off[i + 1]] = g.row_ptr[:-1] + e_off[i]
        col[e_off[i]:e_off[i + 1]] = g.col_idx
    row_ptr[-1] = e_off[-1]
    return GraphBatch(graphs, v_off, e_off, row_ptr, col[: int(e_off[-1])],
                      np.asarray(sources, dtype=np.int32))


def mixed_batch(num: int = 512, seed: int = 5501, rmat_scales=range(10, 19),
                lattice_sides=(128, 256, 512, 1024)) -> GraphBatch:
    """Half R-MAT instances (scale uniform over ``rmat_scales``), half lattice
    instances (side uniform over ``lattice_sides``), in a seeded random order;
    one largest-component source per instance.  Instance i's graph seed is
    derived from (seed, i)."""
    L = _L()
    scales = list(rmat_scales)
    sides = list(lattice_sides)
    kinds = []
    for i in range(num):
        r = L.gg_rng(seed, 8, i)
        if i < num // 2:
            kinds.append(("rmat", scales[r % len(scales)]))
        else:
            kinds.append(("lattice", sides[r % len(sides)]))
    order = np.empty(num, dtype=np.int32)
    L.gg_permutation(num, seed, _p(order))
    graphs, srcs = [], []
    for j in range(num):
        i = int(order[j])
        kind, size = kinds[i]
        gseed = (seed * 1000003 + i) & 0xFFFFFFFF
        g = rmat(size, seed=gseed) if kind == "rmat" else lattice(size, seed=gseed)
        s = pick_sources(g, 1, gseed + 1)
        graphs.append(g)
        srcs.append(int(s[0]))
    return concat(graphs, srcs)


# ---------------------------------------------------------------------------
# the benchmark workloads

def workload(name: str) -> Graph:
    """Named workloads with fixed seeds.

    rmat14   R-MAT scale 14 (16,384 vertices), graph seed 1401
    rmat22   R-MAT scale 22 (4,194,304 vertices), graph seed 2201
    lattice4096  4096^2 lattice with deletions and shortcuts, seed 3301
    er24     Erdos-Renyi, 2^24 vertices, mean degree 8, seed 3401
    """
    if name == "rmat14":
        return rmat(14, seed=1401)
    if name == "rmat22":
        return rmat(22, seed=2201)
    if name == "lattice4096":
        return lattice(4096, seed=3301)
    if name == "er24":
        return erdos_renyi(1 << 24, 8.0, seed=3401)
    if name.startswith("rmat"):
        s = int(name[4:])
        return rmat(s, seed=4000 + s)
    if name.startswith("lattice"):
        side = int(name[7:])
        return lattice(side, seed=4100 + side % 997)
    raise KeyError(name)


WORKLOAD_SOURCES = {"rmat14": (1, 1402), "rmat22": (64, 2202), "lattice4096": (32, 3302),
                    "er24": (32, 3402)}
