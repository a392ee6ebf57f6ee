"""ctypes view of the C ABI in include/bfs_eeds.h (structs, constants,
function signatures).  Loading fails loudly when libbfs_eeds.so is missing:
there is no fallback path."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfs_eeds.so")

BFS_OK = 0
BFS_EINVAL = -1
BFS_EGRAPH = -2
BFS_EWORKSPACE = -3
BFS_EHIP = -4
BFS_ENOSEL = -5
BFS_ELEVELCAP = -6
BFS_ENOTSUP = -7
BFS_EFILE = -8

PUSH_Q_THREAD = 0
PUSH_Q_BLOCK = 1
PUSH_Q_MERGE = 2
PUSH_B_ATOMIC = 3
PUSH_B_NOATOMIC = 4
PUSH_Q_NOATOMIC = 5
PULL_B = 6
PULL_VIS = 7
PUSH_P3 = 8
PUSH_Q_FILTER = 9
PUSH_B_FILTER = 10
PUSH_Q_DEDUP = 11
NUM_VARIANTS = 12
MS_SPLIT = 200  # bfs_multi level_variant: a split bottom-up level
AUTO_HEURISTIC = 100
AUTO_LEARNED = 101
SCHEDULE = 102

VARIANT_NAMES = {
    PUSH_Q_THREAD: "push_q_thread", PUSH_Q_BLOCK: "push_q_block", PUSH_Q_MERGE: "push_q_merge",
    PUSH_B_ATOMIC: "push_b_atomic", PUSH_B_NOATOMIC: "push_b_noatomic",
    PUSH_Q_NOATOMIC: "push_q_noatomic", PULL_B: "pull_b", PULL_VIS: "pull_vis",
    PUSH_P3: "push_p3", PUSH_Q_FILTER: "push_q_filter", PUSH_B_FILTER: "push_b_filter",
    PUSH_Q_DEDUP: "push_q_dedup",
    AUTO_HEURISTIC: "heuristic", AUTO_LEARNED: "learned", SCHEDULE: "schedule",
}

F_VALIDATE = 1
F_STRICT_SELECTOR = 2
F_LEVEL_STATS = 4
F_DEVICE_LOOP = 8
F_LEVEL_TIMING = 16
F_GRAPH_SUMS = 32
F_HUB_ORDER = 64
F_MAIN_TIMING = 128

MLP_NPARAM = 5252
MLP_NFEAT = 12
MLP_NCLASS = 4


class BfsGraph(ctypes.Structure):
    _fields_ = [("n", c_int32), ("nnz", c_int32), ("row_ptr", c_void_p), ("col_idx", c_void_p),
                ("csc_ptr", c_void_p), ("csc_idx", c_void_p)]


class BfsMultiConfig(ctypes.Structure):
    _fields_ = [("wide_ratio", c_int32), ("split_vpt", c_int32), ("cap0", c_int32), ("tile_alpha", c_int32),
                ("alpha", c_int32), ("split_lout", c_int32), ("wide_vpt", c_int32), ("narrow_vpt", c_int32)]


class BfsOptions(ctypes.Structure):
    _fields_ = [("variant", c_int32), ("flags", c_int32), ("schedule_host", POINTER(c_int32)),
                ("schedule_len", c_int32), ("max_levels", c_int32), ("heuristic_push", c_int32),
                ("heuristic_pull", c_int32), ("workspace", c_void_p), ("workspace_bytes", c_size_t),
                ("graph_ld", c_int64), ("graph_ld2", c_int64), ("vertex_map", c_void_p), ("hub_split", c_int32),
                ("multi_config", POINTER(BfsMultiConfig))]


class BfsStats(ctypes.Structure):
    _fields_ = [("num_levels", c_int32), ("fell_back", c_int32), ("reached", c_int64),
                ("component_edges", c_int64), ("elapsed_ms", c_float), ("host_syncs", c_int32),
                ("level_capacity", c_int32), ("level_variant", POINTER(c_int32)),
                ("level_frontier", POINTER(c_int64)), ("level_frontier_edges", POINTER(c_int64)),
                ("level_unvisited", POINTER(c_int64)), ("level_unvisited_edges", POINTER(c_int64)),
                ("level_fallback", POINTER(c_int32)), ("level_frontier_ld", POINTER(c_int64)),
                ("level_frontier_ld2", POINTER(c_int64)), ("graph_ld", c_int64), ("graph_ld2", c_int64),
                ("level_scanned", POINTER(c_int64)), ("level_next", POINTER(c_int64)),
                ("level_ms", POINTER(c_float)), ("level_ms_main", POINTER(c_float)),
                ("level_scanned_aux", POINTER(c_int64)), ("level_hits_aux", POINTER(c_int64)),
                ("level_scanned_push", POINTER(c_int64)), ("level_push_sources", POINTER(c_int64))]


class BfsGraphBatch(ctypes.Structure):
    _fields_ = [("num", c_int32), ("total_n", c_int32), ("total_nnz", c_int32),
                ("v_off_host", POINTER(c_int64)), ("e_off_host", POINTER(c_int64)),
                ("row_ptr", c_void_p), ("col_idx", c_void_p), ("symmetric", c_int32)]


class BfsBatchConfig(ctypes.Structure):
    _fields_ = [("block_threads", c_int32), ("small_vertices", c_int32),
                ("blocks_per_cu", c_int32), ("team_vertices", c_int32), ("max_team", c_int32),
                ("workspace", c_void_p), ("workspace_bytes", c_size_t)]


# name -> (restype, argtypes)
SIGNATURES = {
    "bfs_strerror": (ctypes.c_char_p, [c_int32]),
    "bfs_last_error": (ctypes.c_char_p, []),
    "bfs_version": (c_int32, []),
    "bfs_workspace_size": (c_int32, [c_int32, c_int32, POINTER(c_size_t)]),
    "bfs_reorder_degree": (c_int32, [POINTER(BfsGraph)] + [c_void_p] * 7),
    "bfs_reorder_rcm": (c_int32, [POINTER(BfsGraph)] + [c_void_p] * 7),
    "bfs_graph_sums": (c_int32, [POINTER(BfsGraph), POINTER(c_int64), POINTER(c_int64), c_void_p]),
    "bfs_levels": (c_int32, [POINTER(BfsGraph), c_int32, c_void_p, POINTER(BfsOptions), POINTER(BfsStats),
                             c_void_p]),
    "bfs_parents": (c_int32, [POINTER(BfsGraph), c_int32, c_void_p, c_void_p, POINTER(BfsOptions),
                              POINTER(BfsStats), c_void_p]),
    "bfs_levels_noalloc": (c_int32, [POINTER(BfsGraph), c_int32, c_void_p, POINTER(BfsOptions), POINTER(BfsStats),
                                     c_void_p]),
    "bfs_multi": (c_int32, [POINTER(BfsGraph), POINTER(c_int32), c_int32, c_void_p, POINTER(BfsOptions),
                            POINTER(BfsStats), c_void_p]),
    "bfs_multi_autotune": (c_int32, [POINTER(BfsGraph), POINTER(c_int32), c_int32, c_void_p, POINTER(BfsOptions),
                                     POINTER(BfsMultiConfig), POINTER(c_float), c_void_p]),
    "bfs_batch": (c_int32, [POINTER(BfsGraphBatch), POINTER(c_int32), c_void_p, POINTER(BfsBatchConfig),
                            POINTER(BfsStats), c_void_p]),
    "bfs_batch_autotune": (c_int32, [POINTER(BfsGraphBatch), POINTER(c_int32), c_void_p,
                                     POINTER(BfsBatchConfig), POINTER(c_float), c_void_p]),
    "bfs_batch_workspace_size": (c_int32, [POINTER(BfsGraphBatch), POINTER(c_int32), POINTER(BfsBatchConfig),
                                           POINTER(c_size_t)]),
    "bfs_selector_set": (c_int32, [POINTER(c_float)] * 5 + [c_float, POINTER(c_int32)]),
    "bfs_selector_load": (c_int32, [ctypes.c_char_p]),
    "bfs_selector_clear": (c_int32, []),
    "bfs_selector_loaded": (c_int32, []),
    "bfs_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "bfs_mlp_loss_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "bfs_mlp_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_float, c_float, c_float,
                               c_float, c_void_p]),
    "bfs_mlp_predict": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "bfs_level_features": (c_int32, [POINTER(BfsStats), c_int32, c_int32, POINTER(c_float)]),
    "bfs_step_time": (c_int32, [POINTER(BfsGraph), c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                POINTER(BfsOptions), POINTER(c_float), c_void_p]),
}

_lib = None


class BfsError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: error {code} ({detail})")
        self.code = code


def load() -> ctypes.CDLL:
    """Loads libbfs_eeds.so; raises if it is not built (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2607_17106_amd.build_lib.build() "
                              "(or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int, where: str) -> None:
    if rc != BFS_OK:
        lib = load()
        detail = lib.bfs_last_error().decode(errors="replace")
        raise BfsError(rc, where, f"{lib.bfs_strerror(rc).decode()}: {detail}")
