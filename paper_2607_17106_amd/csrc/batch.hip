// Batched BFS: many independent graphs (a disjoint union stored back to
// back) searched in one persistent launch.
//
// Every workgroup repeatedly takes the next instance from a queue (instances
// ordered largest first, one atomic ticket per instance) and runs that whole
// search by itself, level by level (Cascade 1), with workgroup barriers only.
// Keeping an instance inside one workgroup -- one CU, one XCD L2 -- means its
// visited/frontier state needs no cross-XCD coherence: claims are
// workgroup-scope atomics that resolve in that L2 (or in LDS), and no wait on
// another workgroup ever happens, so the launch always drains.
//
// Per level the workgroup picks a direction from its own counts, comparing
// the in-edges a bottom-up step is expected to read with the frontier's
// out-edges (see the rule in k_batch):
//   top-down: the frontier queue is cut into chunks; each chunk's edges are
//     flattened with a workgroup scan and split evenly over the lanes
//     (Table 3, variant 1 at workgroup scale); a lane claims an unvisited
//     target with an atomicOr on its visited word and appends it.
//   bottom-up (symmetric instances): the frontier queue is scattered into a
//     bitmap; each wave owns 64 consecutive vertices, tests the first in-edges
//     of every unvisited one and scans the rest wave-cooperatively, stopping
//     at the first frontier member.
// Visited and frontier bitmaps live in LDS when the instance is small enough
// (config small_vertices), otherwise in the workgroup's private scratch.
#include <string.h>
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace bfs {

struct BatchArgs {
  int num;
  const int *v_off;   // [num+1]
  const int *order;   // [num] processing order
  const int *src;     // [num] local sources
  const int *rp;      // concatenated CSR: global entry offsets
  const int *ci;      // local column ids
  int *levels;        // [total_n]
  u64 *stats;         // [num][2]: component out-edges, levels
  int *ticket;
  char *scratch;      // per-workgroup slots
  size_t slot_bytes;
  int max_n;
  int small_n;        // LDS bitmaps when n <= small_n
  int chunk;          // frontier vertices per top-down pass
  int symmetric;
};

constexpr int BATCH_T = 4;  // bottom-up: in-edges each lane tests before the wave-cooperative scan

__device__ __forceinline__ u64 or_wg(u64 *p, u64 bits) {
  return __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Frontier-bitmap test: an atomic load at workgroup scope, so it observes the
// workgroup's atomic ORs that precede the last barrier.
__device__ __forceinline__ bool in_frontier(u64 *fr, int u) {
  return (__hip_atomic_load(fr + (u >> 6), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> (u & 63)) & 1ull;
}

template <int BT>
__device__ __forceinline__ int bscan_excl(int x, int *total, int *s_w) {
  const int w = threadIdx.x / WAVE;
  int incl = wave_incl_scan(x);
  if (lane() == WAVE - 1) s_w[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BT / WAVE; ++i) {
    int t = s_w[i];
    off += (i < w) ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

// Appends v (lanes with pred) to q at slots taken from the LDS counter *cnt.
__device__ __forceinline__ void lds_append(bool pred, int v, int *q, int *cnt) {
  const u64 m = __ballot(pred);
  if (!m) return;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane() == leader) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, leader);
  if (pred) q[base + __popcll(m & __lanemask_lt())] = v;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_batch(BatchArgs A) {
  extern __shared__ __align__(16) char dyn[];
  constexpr int CHMAX = 2 * BT;
  __shared__ int s_u[CHMAX], s_off[CHMAX], s_incl[CHMAX], s_w[BT / WAVE];
  __shared__ int s_inst, s_qn;
  __shared__ unsigned long long s_efn;
  u64 *lds_bm = reinterpret_cast<u64 *>(dyn);
  const int lds_words = (A.small_n + 63) / 64;
  const int wv = threadIdx.x / WAVE, nwv = BT / WAVE;
  char *slot = A.scratch + (size_t)blockIdx.x * A.slot_bytes;
  int *qa = reinterpret_cast<int *>(slot);
  int *qb = qa + A.max_n;
  const int max_words = (A.max_n + 63) / 64;
  // the two queues take 8 max_n bytes, rounded up to 256 so that the bitmaps
  // (64-bit atomics) start 256-byte aligned whatever max_n's parity
  u64 *g_vis = reinterpret_cast<u64 *>(slot + (((size_t)A.max_n * 8 + 255) & ~(size_t)255));
  u64 *g_fr = g_vis + max_words;
  for (;;) {
    if (threadIdx.x == 0) s_inst = atomicAdd(A.ticket, 1);
    __syncthreads();
    const int t = s_inst;
    __syncthreads();
    if (t >= A.num) break;
    const int b = A.order[t];
    const int V0 = A.v_off[b];
    const int n = A.v_off[b + 1] - V0;
    const int *rp = A.rp + V0;
    int *lv = A.levels + V0;
    const int W = (n + 63) / 64;
    const bool small = n <= A.small_n;
    u64 *vis = small ? lds_bm : g_vis;
    u64 *fr = small ? lds_bm + lds_words : g_fr;
    int *qc = qa, *qn = qb;
    const int src = A.src[b];
    // ---- init
    for (int v = threadIdx.x; v < n; v += BT) lv[v] = (v == src) ? 0 : -1;
    for (int w = threadIdx.x; w < W; w += BT) {
      u64 x = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
      if (w == W - 1 && (n & 63)) x |= ~0ull << (n & 63);
      vis[w] = x;
    }
    if (threadIdx.x == 0) {
      qc[0] = src;
      s_qn = 1;
      s_efn = (unsigned long long)(rp[src + 1] - rp[src]);
    }
    __syncthreads();
    long long nF = s_qn, eF = (long long)s_efn;
    long long eU = (long long)(rp[n] - rp[0]) - eF;
    long long nU = n - 1;
    long long comp = eF;
    int dir = 0;
    int k = 0;
    for (;; ++k) {
      if (A.symmetric) {
        // One workgroup pays for every in-edge a bottom-up step reads.  An
        // unvisited vertex reads about (e_U + e_F) / e_F in-edges before it
        // meets a frontier member (in-edges drawn at random), and at most its
        // degree, so the step reads about min(e_U, n_U (e_U + e_F) / e_F);
        // the top-down step reads e_F.
        const long long scan = eF > 0 ? min(eU, nU * ((eU + eF) / eF + 1)) : eU;
        dir = scan < eF ? 1 : 0;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        s_qn = 0;
        s_efn = 0ull;
      }
      __syncthreads();
      u64 my_efn = 0;  // out-edges of the vertices this thread discovers (reduced per wave below)
      if (dir == 0) {
        // ---- top-down over the frontier queue, flattened chunk by chunk
        const int CH = A.chunk;
        for (int c0 = 0; c0 < nF; c0 += CH) {
          const int per = CH / BT;
          int run = 0, deg[2], beg[2], uu[2];
          for (int r = 0; r < per; ++r) {
            const int i = c0 + threadIdx.x * per + r;
            int u = -1, d = 0, bg = 0;
            if (i < nF) {
              u = qc[i];
              bg = rp[u];
              d = rp[u + 1] - bg;
            }
            run += d;
            deg[r] = run;
            beg[r] = bg;
            uu[r] = u;
          }
          int total;
          const int off = bscan_excl<BT>(run, &total, s_w);
          for (int r = 0; r < per; ++r) {
            const int j = threadIdx.x * per + r;
            const int inc = off + deg[r];
            const int d = deg[r] - (r ? deg[r - 1] : 0);
            s_incl[j] = inc;
            s_u[j] = uu[r];
            s_off[j] = beg[r] - (inc - d);
          }
          __syncthreads();
          for (int e = threadIdx.x; e < total; e += BT) {
            int lo = 0, hi = CH - 1;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (s_incl[mid] > e) hi = mid; else lo = mid + 1;
            }
            const int v = A.ci[s_off[lo] + e];
            const u64 bit = 1ull << (v & 63);
            bool win = false;
            if (!(vis[v >> 6] & bit)) win = !(or_wg(vis + (v >> 6), bit) & bit);
            if (win) {
              lv[v] = k + 1;
              my_efn += (u64)(rp[v + 1] - rp[v]);
            }
            lds_append(win, v, qn, &s_qn);
          }
          __syncthreads();
        }
      } else {
        // ---- bottom-up: frontier bitmap from the queue, then one wave per word
        for (int w = threadIdx.x; w < W; w += BT) fr[w] = 0ull;
        __syncthreads();
        for (int i = threadIdx.x; i < nF; i += BT) {
          const int u = qc[i];
          or_wg(fr + (u >> 6), 1ull << (u & 63));
        }
        __syncthreads();
        for (int w = wv; w < W; w += nwv) {
          const u64 vw = vis[w];
          if (vw == ~0ull) continue;
          const int v = w * WAVE + lane();
          bool found = false, pending = false;
          int bb = 0, ee = 0;
          if (!((vw >> lane()) & 1ull)) {
            bb = rp[v];
            ee = rp[v + 1];
            const int d = ee - bb;
            for (int t2 = 0; t2 < BATCH_T && t2 < d && !found; ++t2) {
              found = in_frontier(fr, A.ci[bb + t2]);
            }
            pending = !found && d > BATCH_T;
            bb += BATCH_T;
          }
          u64 pm = __ballot(pending);
          while (pm) {
            const int l = __ffsll((long long)pm) - 1;
            pm &= pm - 1;
            const int vb = __shfl(bb, l), ve = __shfl(ee, l);
            for (int base = vb; base < ve; base += WAVE) {
              const int j = base + lane();
              bool hit = false;
              if (j < ve) hit = in_frontier(fr, A.ci[j]);
              if (__ballot(hit)) {
                if (lane() == l) found = true;
                break;
              }
            }
          }
          const u64 m = __ballot(found);
          if (m) {
            if (lane() == 0) vis[w] = vw | m;
            if (found) {
              lv[v] = k + 1;
              my_efn += (u64)(rp[v + 1] - rp[v]);
            }
            lds_append(found, v, qn, &s_qn);
          }
        }
      }
      {
        const u64 we = wave_sum_u64(my_efn);
        if (lane() == 0 && we) atomicAdd(&s_efn, (unsigned long long)we);
      }
      __syncthreads();
      nF = s_qn;
      eF = (long long)s_efn;
      eU -= eF;  // symmetric instances: in-edges = out-edges of the new vertices
      nU -= nF;
      comp += eF;
      int *tq = qc;
      qc = qn;
      qn = tq;
      if (nF == 0) break;
    }
    if (threadIdx.x == 0) {
      A.stats[2 * b] = (u64)comp;
      A.stats[2 * b + 1] = (u64)(k + 1);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- host
static int cus_of_device() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

static bool config_ok(const bfs_batch_config &c) {
  if (c.block_threads != 256 && c.block_threads != 512 && c.block_threads != 1024) return false;
  if (c.blocks_per_cu < 1 || c.blocks_per_cu > 4) return false;
  if (c.chunk_vertices < c.block_threads || c.chunk_vertices > 2 * c.block_threads ||
      c.chunk_vertices % c.block_threads)
    return false;
  if (c.small_vertices < 0 || c.small_vertices > (1 << 18)) return false;
  return true;
}

static bfs_batch_config default_config() {
  bfs_batch_config c;
  c.block_threads = 512;
  c.small_vertices = 65536;
  c.chunk_vertices = 512;
  c.blocks_per_cu = 2;
  return c;
}

struct BatchPlan {
  int grid;
  size_t slot_bytes;
  int max_n;
};

static std::mutex g_tune_mu;
static std::map<std::tuple<int, long long, long long>, bfs_batch_config> g_tuned;

// Device scratch: [v_off | order | src | ticket] ints, stats, slots.
static int batch_run(const bfs_graph_batch *b, const int32_t *sources, int32_t *levels, const bfs_batch_config &cfg,
                     bfs_stats *st, hipStream_t s, float *ms_out) {
  const int num = b->num;
  std::vector<int> voff(num + 1), order(num);
  int max_n = 0;
  for (int i = 0; i <= num; ++i) voff[i] = (int)b->v_off_host[i];
  for (int i = 0; i < num; ++i) max_n = std::max(max_n, voff[i + 1] - voff[i]);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    long long cx = (b->e_off_host[x + 1] - b->e_off_host[x]) + (voff[x + 1] - voff[x]);
    long long cy = (b->e_off_host[y + 1] - b->e_off_host[y]) + (voff[y + 1] - voff[y]);
    return cx > cy;
  });
  const int cus = cus_of_device();
  if (cus <= 0) return hip_fail(hipErrorInvalidDevice, "hipDeviceGetAttribute(multiProcessorCount)");
  const int grid = std::min(num, cfg.blocks_per_cu * cus);
  size_t ints = (size_t)(num + 1) + 2 * (size_t)num + 64;
  size_t head = ((ints * 4 + 255) & ~(size_t)255) + (((size_t)num * 16 + 255) & ~(size_t)255);
  size_t slot = (((size_t)max_n * 8 + 255) & ~(size_t)255) + 2 * (size_t)((max_n + 63) / 64) * 8;
  slot = (slot + 255) & ~(size_t)255;
  void *wsp = nullptr;
  int rc = cached_workspace(head + slot * (size_t)grid, &wsp);
  if (rc) return rc;
  char *p = (char *)wsp;
  int *d_voff = (int *)p, *d_order = d_voff + num + 1, *d_src = d_order + num, *d_ticket = d_src + num;
  u64 *d_stats = (u64 *)(p + ((ints * 4 + 255) & ~(size_t)255));
  char *d_slots = p + head;
  std::vector<int> hostbuf(ints, 0);
  memcpy(hostbuf.data(), voff.data(), (num + 1) * 4);
  memcpy(hostbuf.data() + num + 1, order.data(), num * 4);
  memcpy(hostbuf.data() + 2 * num + 1, sources, num * 4);
  HostCtx &hc = host_ctx();
  BFS_HIP(hipMemcpyAsync(d_voff, hostbuf.data(), ints * 4, hipMemcpyHostToDevice, s));
  BatchArgs A;
  A.num = num;
  A.v_off = d_voff;
  A.order = d_order;
  A.src = d_src;
  A.rp = b->row_ptr;
  A.ci = b->col_idx;
  A.levels = levels;
  A.stats = d_stats;
  A.ticket = d_ticket;
  A.scratch = d_slots;
  A.slot_bytes = slot;
  A.max_n = max_n;
  A.small_n = cfg.small_vertices;
  A.chunk = cfg.chunk_vertices;
  A.symmetric = b->symmetric ? 1 : 0;
  const size_t lds = 2 * (size_t)((cfg.small_vertices + 63) / 64) * 8;
  BFS_HIP(hipEventRecord(hc.ev[2], s));
  switch (cfg.block_threads) {
    case 256: hipLaunchKernelGGL(k_batch<256>, dim3(grid), dim3(256), lds, s, A); break;
    case 512: hipLaunchKernelGGL(k_batch<512>, dim3(grid), dim3(512), lds, s, A); break;
    default: hipLaunchKernelGGL(k_batch<1024>, dim3(grid), dim3(1024), lds, s, A); break;
  }
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipEventRecord(hc.ev[3], s));
  std::vector<u64> stats((size_t)num * 2);
  BFS_HIP(hipMemcpyAsync(stats.data(), d_stats, num * 16, hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  BFS_HIP(hipEventElapsedTime(&ms, hc.ev[2], hc.ev[3]));
  if (ms_out) *ms_out = ms;
  if (st) {
    long long comp = 0, lev = 0;
    for (int i = 0; i < num; ++i) {
      comp += (long long)stats[2 * i];
      lev = std::max(lev, (long long)stats[2 * i + 1]);
    }
    st->component_edges = comp;
    st->num_levels = (int)lev;
    st->elapsed_ms = ms;
    st->host_syncs = 1;
    st->reached = -1;  // not counted by the batched kernel
  }
  return BFS_OK;
}

static int check_batch(const bfs_graph_batch *b, const int32_t *sources, const int32_t *levels) {
  if (!b || b->num <= 0 || !b->v_off_host || !b->e_off_host || !b->row_ptr || !sources || !levels ||
      (!b->col_idx && b->total_nnz > 0)) {
    set_error("bfs_batch: invalid argument");
    return BFS_EINVAL;
  }
  if (b->v_off_host[0] != 0 || b->v_off_host[b->num] != b->total_n || b->e_off_host[0] != 0 ||
      b->e_off_host[b->num] != b->total_nnz) {
    set_error("bfs_batch: offsets do not span total_n / total_nnz");
    return BFS_EINVAL;
  }
  for (int i = 0; i < b->num; ++i) {
    const long long n = b->v_off_host[i + 1] - b->v_off_host[i];
    if (n <= 0 || b->e_off_host[i + 1] < b->e_off_host[i]) {
      set_error("bfs_batch: instance %d is empty or has negative edge range", i);
      return BFS_EINVAL;
    }
    if (sources[i] < 0 || sources[i] >= n) {
      set_error("bfs_batch: source %d of instance %d out of range", sources[i], i);
      return BFS_EINVAL;
    }
  }
  return BFS_OK;
}

}  // namespace bfs

using namespace bfs;

extern "C" int bfs_batch(const bfs_graph_batch *b, const int32_t *sources, int32_t *levels,
                         const bfs_batch_config *cfg_in, bfs_stats *st, void *stream) {
  int rc = check_batch(b, sources, levels);
  if (rc) return rc;
  bfs_batch_config cfg = default_config();
  if (cfg_in) {
    cfg = *cfg_in;
  } else {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(b->num, (long long)b->total_n, (long long)b->total_nnz));
    if (it != g_tuned.end()) cfg = it->second;
  }
  if (!config_ok(cfg)) {
    set_error("bfs_batch: invalid config (threads %d, blocks/CU %d, chunk %d, small %d)", cfg.block_threads,
              cfg.blocks_per_cu, cfg.chunk_vertices, cfg.small_vertices);
    return BFS_EINVAL;
  }
  return batch_run(b, sources, levels, cfg, st, (hipStream_t)stream, nullptr);
}

extern "C" int bfs_batch_autotune(const bfs_graph_batch *b, const int32_t *sources, int32_t *levels,
                                  bfs_batch_config *best, float *ms_best, void *stream) {
  int rc = check_batch(b, sources, levels);
  if (rc) return rc;
  if (!best) {
    set_error("bfs_batch_autotune: best is NULL");
    return BFS_EINVAL;
  }
  float best_ms = 1e30f;
  bfs_batch_config bc = default_config();
  for (int bt : {256, 512, 1024})
    for (int bpc : {1, 2, 4})
      for (int small : {0, 16384, 65536, 131072})
        for (int chm : {1, 2}) {
          bfs_batch_config c;
          c.block_threads = bt;
          c.blocks_per_cu = bpc;
          c.small_vertices = small;
          c.chunk_vertices = chm * bt;
          if (!config_ok(c)) continue;
          if ((size_t)small / 4 + 3 * 2 * bt * 4 > 64 * 1024 && bpc > 2) continue;  // LDS budget
          float t = 0.f, ms;
          rc = batch_run(b, sources, levels, c, nullptr, (hipStream_t)stream, &ms);  // warm-up
          if (rc) return rc;
          rc = batch_run(b, sources, levels, c, nullptr, (hipStream_t)stream, &ms);
          if (rc) return rc;
          t = ms;
          if (t < best_ms) {
            best_ms = t;
            bc = c;
          }
        }
  *best = bc;
  if (ms_best) *ms_best = best_ms;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[std::make_tuple(b->num, (long long)b->total_n, (long long)b->total_nnz)] = bc;
  return BFS_OK;
}
