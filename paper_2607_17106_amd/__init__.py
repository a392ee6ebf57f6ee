"""MI355X-native BFS level step over int32 CSR/CSC (see include/bfs_eeds.h).

Python binding: argument marshalling only.  Every step of the search runs in
the HIP kernels of libbfs_eeds.so; PyTorch supplies device memory and the
stream.  Importing this package does not load the library; the first call
does, and fails loudly when it is not built.
"""
from ._lib import (  # noqa: F401
    PUSH_Q_THREAD, PUSH_Q_BLOCK, PUSH_Q_MERGE, PUSH_B_ATOMIC, PUSH_B_NOATOMIC, PUSH_Q_NOATOMIC, PULL_B, PULL_VIS, PUSH_P3, PUSH_Q_FILTER, PUSH_B_FILTER,
    PUSH_Q_DEDUP,
    NUM_VARIANTS, MS_SPLIT, AUTO_HEURISTIC, AUTO_LEARNED, SCHEDULE, VARIANT_NAMES, F_VALIDATE, F_STRICT_SELECTOR,
    F_LEVEL_STATS, F_DEVICE_LOOP, F_LEVEL_TIMING, F_GRAPH_SUMS, F_HUB_ORDER, F_MAIN_TIMING, BfsError, load,
)
from .api import (  # noqa: F401
    DeviceGraph, DeviceBatch, bfs_levels, bfs_levels_noalloc, bfs_parents, bfs_multi, bfs_multi_autotune,
    MultiConfig, bfs_batch, bfs_batch_autotune,
    workspace_size, selector_set, selector_clear, selector_loaded, mlp_forward, mlp_loss_grad, mlp_adam,
    mlp_predict, level_features, step_time, reorder_degree, reorder_rcm,
)
