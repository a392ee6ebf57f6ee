#include "common.hpp"
extern "C" {
int bfs_batch(const bfs_graph_batch *, const int32_t *, int32_t *, const bfs_batch_config *, bfs_stats *, void *) { return BFS_ENOTSUP; }
int bfs_batch_autotune(const bfs_graph_batch *, const int32_t *, int32_t *, bfs_batch_config *, float *, void *) { return BFS_ENOTSUP; }
}
