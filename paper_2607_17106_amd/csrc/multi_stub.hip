#include "common.hpp"
namespace bfs {
size_t workspace_bytes_multi(int n) { return (size_t)n * 8 * 4 + 4096; }
}
extern "C" {
int bfs_multi(const bfs_graph *, const int32_t *, int32_t, int32_t *, const bfs_options *, bfs_stats *, void *) { return BFS_ENOTSUP; }
int bfs_batch(const bfs_graph_batch *, const int32_t *, int32_t *, const bfs_batch_config *, bfs_stats *, void *) { return BFS_ENOTSUP; }
int bfs_batch_autotune(const bfs_graph_batch *, const int32_t *, int32_t *, bfs_batch_config *, float *, void *) { return BFS_ENOTSUP; }
}
