// Vertex renumbering, a preprocessing step: by decreasing out-degree, or
// reverse Cuthill-McKee (the paper renumbers every graph with the latter
// before timing; Sec. "Experiment Setup", its preprocessing paragraph).
//
// The degree order puts vertices of high out-degree first.  In a bottom-up step
// every in-edge (u, v) reads the frontier state of u, and u appears in as many
// in-edge lists as it has out-edges: after the renumbering the states read
// most often share a few hundred KB of cache lines, and each ascending in-edge
// list starts with its most connected in-neighbours, which are the likeliest
// to be in the frontier, so the early exit comes sooner.
//
// Order: new id i holds the vertex with the i-th largest out-degree, ties in
// increasing old id.  Both are the ascending order of the unique 64-bit keys
// (INT32_MAX - outdeg) << 32 | id.  The renumbered CSR (and CSC) are the
// ascending order of the keys new(u) << b | new(v) over the edges, b the bits
// of n - 1; row i's length is that of old row old_of_new[i], so the offsets
// are a scan of the permuted lengths.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <vector>

#include "common.hpp"

namespace bfs {
namespace {

__global__ __launch_bounds__(BLOCK) void k_vertex_keys(const int *rp, int n, u64 *keys) {
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < n; v += gridDim.x * BLOCK)
    keys[v] = ((u64)(u32)(0x7fffffffll - (rp[v + 1] - rp[v])) << 32) | (u64)(u32)v;
}

__global__ __launch_bounds__(BLOCK) void k_vertex_perm(const u64 *keys, int n, int *new_of_old, int *old_of_new) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    const int old = (int)(u32)keys[i];
    old_of_new[i] = old;
    new_of_old[old] = i;
  }
}

// lens[i] = length of old row old_of_new[i]; lens[n] = 0 (the scan's total slot)
__global__ __launch_bounds__(BLOCK) void k_row_lens(const int *ptr, const int *old_of_new, int n, int *lens) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i <= n; i += gridDim.x * BLOCK) {
    if (i < n) {
      const int o = old_of_new[i];
      lens[i] = ptr[o + 1] - ptr[o];
    } else {
      lens[n] = 0;
    }
  }
}

// One wave per old row u: its entries become new(u) << b | new(idx[j]), in place.
__global__ __launch_bounds__(BLOCK) void k_edge_keys(const int *ptr, const int *idx, int n, const int *new_of_old,
                                                     int b, u64 *keys) {
  const int waves = gridDim.x * (BLOCK / WAVE);
  for (int u = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE; u < n; u += waves) {
    const int e0 = ptr[u], e1 = ptr[u + 1];
    const u64 hi = (u64)new_of_old[u] << b;
    for (int j = e0 + lane(); j < e1; j += WAVE) keys[j] = hi | (u64)(u32)new_of_old[idx[j]];
  }
}

__global__ __launch_bounds__(BLOCK) void k_edge_cols(const u64 *keys, long long nnz, u64 mask, int *idx) {
  for (long long e = blockIdx.x * (long long)BLOCK + threadIdx.x; e < nnz; e += (long long)gridDim.x * BLOCK)
    idx[e] = (int)(keys[e] & mask);
}

int grid_for(long long items) { return (int)std::max(1ll, std::min(8192ll, (items + BLOCK - 1) / BLOCK)); }

struct Temp {
  void *p = nullptr;
  ~Temp() {
    if (p) (void)hipFree(p);
  }
};

// Device temporaries of a renumbering: two key buffers of max(n, nnz) words,
// the row lengths, the rocPRIM scratch of the largest sort and scan, and the
// validation flag.  Frees itself.
struct Scratch {
  Temp tmp;
  u64 *k0 = nullptr, *k1 = nullptr, *flag = nullptr;
  int *lens = nullptr;
  void *sort_tmp = nullptr, *scan_tmp = nullptr;
  size_t sort_bytes = 0, scan_bytes = 0;
  int b = 1;  // bits of n - 1 (at least 1)

  int init(int n, int nnz, hipStream_t s) {
    while (b < 31 && (1ll << b) < (long long)n) ++b;
    const size_t words = std::max<size_t>((size_t)n, (size_t)nnz);
    size_t vsort_bytes = 0;
    rocprim::double_buffer<u64> db(nullptr, nullptr);
    BFS_HIP(rocprim::radix_sort_keys(nullptr, sort_bytes, db, (size_t)std::max(nnz, 1), 0, 2 * b, s));
    BFS_HIP(rocprim::radix_sort_keys(nullptr, vsort_bytes, db, (size_t)n, 0, 64, s));
    BFS_HIP(rocprim::exclusive_scan(nullptr, scan_bytes, (int *)nullptr, (int *)nullptr, 0, (size_t)n + 1,
                                    rocprim::plus<int>(), s));
    const auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    sort_bytes = std::max(sort_bytes, vsort_bytes);
    const size_t total = 2 * al(words * 8) + al(((size_t)n + 1) * 4) + al(sort_bytes) + al(scan_bytes) + 256;
    BFS_HIP(hipMalloc(&tmp.p, total));
    char *p = static_cast<char *>(tmp.p);
    k0 = reinterpret_cast<u64 *>(p);
    k1 = reinterpret_cast<u64 *>(p + al(words * 8));
    lens = reinterpret_cast<int *>(p + 2 * al(words * 8));
    sort_tmp = p + 2 * al(words * 8) + al(((size_t)n + 1) * 4);
    scan_tmp = static_cast<char *>(sort_tmp) + al(sort_bytes);
    flag = reinterpret_cast<u64 *>(p + total - 256);
    return BFS_OK;
  }
};

// RCM degree keys: deg << 32 | id, deg counting out-edges and, for a graph
// with its own CSC, in-edges (the undirected structure).
__global__ __launch_bounds__(BLOCK) void k_rcm_keys(const int *rp, const int *cp, int n, u64 *keys) {
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < n; v += gridDim.x * BLOCK) {
    long long d = rp[v + 1] - rp[v];
    if (cp) d += cp[v + 1] - cp[v];
    keys[v] = ((u64)d << 32) | (u64)(u32)v;
  }
}

// One adjacency (CSR or CSC) renumbered: out_ptr [n+1], out_idx [nnz].
int relabel_adjacency(const int *ptr, const int *idx, int n, int nnz, const int *new_of_old, const int *old_of_new,
                      int *out_ptr, int *out_idx, u64 *k0, u64 *k1, int *lens, void *sort_tmp, size_t sort_bytes,
                      void *scan_tmp, size_t scan_bytes, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_row_lens, dim3(grid_for((long long)n + 1)), dim3(BLOCK), 0, s, ptr, old_of_new, n, lens);
  BFS_HIP(hipGetLastError());
  BFS_HIP(rocprim::exclusive_scan(scan_tmp, scan_bytes, lens, out_ptr, 0, (size_t)n + 1, rocprim::plus<int>(), s));
  if (nnz == 0) return BFS_OK;
  hipLaunchKernelGGL(k_edge_keys, dim3(std::max(1, std::min(16384, (n + 3) / 4))), dim3(BLOCK), 0, s, ptr, idx, n,
                     new_of_old, b, k0);
  BFS_HIP(hipGetLastError());
  rocprim::double_buffer<u64> db(k0, k1);
  BFS_HIP(rocprim::radix_sort_keys(sort_tmp, sort_bytes, db, (size_t)nnz, 0, 2 * b, s));
  hipLaunchKernelGGL(k_edge_cols, dim3(grid_for(nnz)), dim3(BLOCK), 0, s, (const u64 *)db.current(), (long long)nnz,
                     (u64)((1ull << b) - 1), out_idx);
  BFS_HIP(hipGetLastError());
  return BFS_OK;
}

}  // namespace

// Vertices ordered by the unique keys k0[0 .. n) (radix-sorted ascending):
// new_of_old / old_of_new from the ids in their low 32 bits.
static int order_from_keys(Scratch &t, int n, int *new_of_old, int *old_of_new, hipStream_t s) {
  rocprim::double_buffer<u64> db(t.k0, t.k1);
  BFS_HIP(rocprim::radix_sort_keys(t.sort_tmp, t.sort_bytes, db, (size_t)n, 0, 64, s));
  hipLaunchKernelGGL(k_vertex_perm, dim3(grid_for(n)), dim3(BLOCK), 0, s, (const u64 *)db.current(), n, new_of_old,
                     old_of_new);
  BFS_HIP(hipGetLastError());
  return BFS_OK;
}

// The CSR (and the CSC, when the graph has its own) renumbered by the maps.
static int relabel_graph(Scratch &t, const bfs_graph *g, const int *new_of_old, const int *old_of_new,
                         int *out_row_ptr, int *out_col_idx, int *out_csc_ptr, int *out_csc_idx, hipStream_t s) {
  int rc = relabel_adjacency(g->row_ptr, g->col_idx, g->n, g->nnz, new_of_old, old_of_new, out_row_ptr, out_col_idx,
                             t.k0, t.k1, t.lens, t.sort_tmp, t.sort_bytes, t.scan_tmp, t.scan_bytes, t.b, s);
  if (rc) return rc;
  if (g->csc_ptr && g->csc_ptr != g->row_ptr)
    rc = relabel_adjacency(g->csc_ptr, g->csc_idx, g->n, g->nnz, new_of_old, old_of_new, out_csc_ptr, out_csc_idx,
                           t.k0, t.k1, t.lens, t.sort_tmp, t.sort_bytes, t.scan_tmp, t.scan_bytes, t.b, s);
  return rc;
}

int reorder_degree(const bfs_graph *g, int *out_row_ptr, int *out_col_idx, int *out_csc_ptr, int *out_csc_idx,
                   int *new_of_old, int *old_of_new, hipStream_t s) {
  const int n = g->n;
  Scratch t;
  int rc = t.init(n, g->nnz, s);
  if (rc) return rc;
  // offsets and ids are checked first: the passes below index by them
  rc = validate_graph(g, t.flag, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_vertex_keys, dim3(grid_for(n)), dim3(BLOCK), 0, s, g->row_ptr, n, t.k0);
  BFS_HIP(hipGetLastError());
  rc = order_from_keys(t, n, new_of_old, old_of_new, s);
  if (rc) return rc;
  rc = relabel_graph(t, g, new_of_old, old_of_new, out_row_ptr, out_col_idx, out_csc_ptr, out_csc_idx, s);
  if (rc) return rc;
  BFS_HIP(hipStreamSynchronize(s));  // the temporaries are freed on return
  return BFS_OK;
}

// Reverse Cuthill-McKee.  Vertices are ranked by (deg, id), deg counting the
// undirected structure (out-edges, plus in-edges when the graph has its own
// CSC).  In the graph renumbered by rank (built on the GPU, rows ascending)
// Cuthill-McKee is one pass on the host: each component starts at the
// smallest unvisited rank, and a visited vertex's unvisited neighbours are
// appended in ascending rank, i.e. in (deg, id) order (its CSR and CSC rows
// merged).  The order is reversed and the graph renumbered by it on the GPU.
int reorder_rcm(const bfs_graph *g, int *out_row_ptr, int *out_col_idx, int *out_csc_ptr, int *out_csc_idx,
                int *new_of_old, int *old_of_new, hipStream_t s) {
  const int n = g->n, nnz = g->nnz;
  const bool csc = g->csc_ptr && g->csc_ptr != g->row_ptr;
  Scratch t;
  int rc = t.init(n, nnz, s);
  if (rc) return rc;
  rc = validate_graph(g, t.flag, s);
  if (rc) return rc;
  // rank maps (held in the output maps until the end) and the rank-space graph
  hipLaunchKernelGGL(k_rcm_keys, dim3(grid_for(n)), dim3(BLOCK), 0, s, g->row_ptr, csc ? g->csc_ptr : nullptr, n,
                     t.k0);
  BFS_HIP(hipGetLastError());
  rc = order_from_keys(t, n, new_of_old, old_of_new, s);
  if (rc) return rc;
  rc = relabel_graph(t, g, new_of_old, old_of_new, out_row_ptr, out_col_idx, out_csc_ptr, out_csc_idx, s);
  if (rc) return rc;
  std::vector<int> rp((size_t)n + 1), ci((size_t)std::max(nnz, 1)), cp, cx, old_of_rank((size_t)n);
  BFS_HIP(hipMemcpyAsync(rp.data(), out_row_ptr, ((size_t)n + 1) * 4, hipMemcpyDeviceToHost, s));
  if (nnz) BFS_HIP(hipMemcpyAsync(ci.data(), out_col_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  if (csc) {
    cp.resize((size_t)n + 1);
    cx.resize((size_t)std::max(nnz, 1));
    BFS_HIP(hipMemcpyAsync(cp.data(), out_csc_ptr, ((size_t)n + 1) * 4, hipMemcpyDeviceToHost, s));
    if (nnz) BFS_HIP(hipMemcpyAsync(cx.data(), out_csc_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  }
  BFS_HIP(hipMemcpyAsync(old_of_rank.data(), old_of_new, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  // Cuthill-McKee in rank space
  std::vector<char> seen((size_t)n, 0);
  std::vector<int> order;
  order.reserve((size_t)n);
  int start = 0;
  while ((int)order.size() < n) {
    while (seen[(size_t)start]) ++start;
    seen[(size_t)start] = 1;
    order.push_back(start);
    for (size_t head = order.size() - 1; head < order.size(); ++head) {
      const int u = order[head];
      int i = rp[(size_t)u], ie = rp[(size_t)u + 1];
      int j = csc ? cp[(size_t)u] : 0, je = csc ? cp[(size_t)u + 1] : 0;
      while (i < ie || j < je) {  // both rows ascending: merge
        int w;
        if (j >= je || (i < ie && ci[(size_t)i] <= cx[(size_t)j]))
          w = ci[(size_t)i++];
        else
          w = cx[(size_t)j++];
        if (!seen[(size_t)w]) {
          seen[(size_t)w] = 1;
          order.push_back(w);
        }
      }
    }
  }
  std::vector<int> o2n((size_t)n), n2o((size_t)n);
  for (int i = 0; i < n; ++i) {
    const int old = old_of_rank[(size_t)order[(size_t)(n - 1 - i)]];
    o2n[(size_t)i] = old;
    n2o[(size_t)old] = i;
  }
  BFS_HIP(hipMemcpyAsync(old_of_new, o2n.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  BFS_HIP(hipMemcpyAsync(new_of_old, n2o.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  rc = relabel_graph(t, g, new_of_old, old_of_new, out_row_ptr, out_col_idx, out_csc_ptr, out_csc_idx, s);
  if (rc) return rc;
  BFS_HIP(hipStreamSynchronize(s));  // host vectors and device temporaries are freed on return
  return BFS_OK;
}

}  // namespace bfs

static int reorder_entry(const char *name, int (*fn)(const bfs_graph *, int *, int *, int *, int *, int *, int *,
                                                    hipStream_t),
                         const bfs_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx, int32_t *out_csc_ptr,
                         int32_t *out_csc_idx, int32_t *new_of_old, int32_t *old_of_new, void *stream) {
  using namespace bfs;
  if (!g || g->n <= 0 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && !g->col_idx) || !out_row_ptr ||
      (g->nnz > 0 && !out_col_idx) || !new_of_old || !old_of_new) {
    set_error("%s: invalid argument", name);
    return BFS_EINVAL;
  }
  const bool csc = g->csc_ptr && g->csc_ptr != g->row_ptr;
  if (csc && (!g->csc_idx || !out_csc_ptr || (g->nnz > 0 && !out_csc_idx))) {
    set_error("%s: a graph with its own CSC needs out_csc_ptr and out_csc_idx", name);
    return BFS_EINVAL;
  }
  return fn(g, out_row_ptr, out_col_idx, out_csc_ptr, out_csc_idx, new_of_old, old_of_new, (hipStream_t)stream);
}

extern "C" int bfs_reorder_degree(const bfs_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx,
                                  int32_t *out_csc_ptr, int32_t *out_csc_idx, int32_t *new_of_old,
                                  int32_t *old_of_new, void *stream) {
  return reorder_entry("bfs_reorder_degree", bfs::reorder_degree, g, out_row_ptr, out_col_idx, out_csc_ptr,
                       out_csc_idx, new_of_old, old_of_new, stream);
}

extern "C" int bfs_reorder_rcm(const bfs_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx, int32_t *out_csc_ptr,
                               int32_t *out_csc_idx, int32_t *new_of_old, int32_t *old_of_new, void *stream) {
  return reorder_entry("bfs_reorder_rcm", bfs::reorder_rcm, g, out_row_ptr, out_col_idx, out_csc_ptr, out_csc_idx,
                       new_of_old, old_of_new, stream);
}
