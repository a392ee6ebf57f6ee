// Multi-source BFS with up to 64 bit-packed lanes per vertex.
//
// Cascade 1 starts from "the source node(s)" (its initialisation); giving F
// and P one more rank for the source index and packing 64 of its coordinates
// into one u64 per vertex turns a level into word-wide boolean algebra:
//   next[v] = (OR_{u in N_in(v)} front[u]) AND NOT vis[v]     (advance, pull)
//   vis[v]  = vis[v] OR next[v]                                (update)
// and depth k+1 is recorded for every lane bit newly set at v.
//
// Pull (bottom-up, CSC): one wave per 64 consecutive vertices; a lane ORs the
// frontier words of its first MS_T in-neighbours, then vertices still needing
// lanes are scanned by the whole wave, 64 in-edges per iteration with an OR
// reduction, stopping once every lane the vertex lacks has been found.
// Push (top-down, CSR): frontier vertices OR their frontier word, masked by
// the target's (read-only) visited word, into the target's next word with
// atomicOr; an owner-computes pass then applies the update.
// Depth rows are written exactly once: at discovery, or -1 by a final pass.
#include <string.h>
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "selector.hpp"

namespace bfs {

constexpr int MS_T = 4;

struct MsCtr {  // one 64-byte line per shard
  u64 newbits;     // (lane, vertex) pairs discovered
  u64 comp_edges;  // sum over discoveries of outdeg(v) (per lane)
  u64 active;      // vertices with at least one new lane (next frontier size)
  u64 active_out;  // their out-edges
  u64 done_in;     // in-edges of vertices whose last lane was found
  u64 scanned;     // edges examined
  u64 pad[2];
};
static_assert(sizeof(MsCtr) == 64, "MsCtr is one line");

struct MsArgs {
  int n, k, L;          // vertices, level, lanes in this group
  u64 full;             // mask of the L lanes
  const int *rp, *ci, *cp, *cx;
  const u64 *front;     // F_k words
  u64 *next;            // F_{k+1} words
  u64 *dead;            // buffer to clear for F_{k+2}
  u64 *vis;
  int *levels;          // row l at levels + l * n
  MsCtr *sh;            // NSH shards of this level's counters
};

size_t workspace_bytes_multi(int n) {
  size_t b = 4 * (((size_t)n * 8 + 255) & ~(size_t)255);  // front[3], vis
  b += (size_t)(NSH + 1) * sizeof(MsCtr) + 512;          // shards, total, sources, degrees
  return b;
}

__device__ __forceinline__ void ms_write_levels(const MsArgs &a, int v, u64 bits, int val) {
  while (bits) {
    const int l = __ffsll((long long)bits) - 1;
    bits &= bits - 1;
    a.levels[(size_t)l * a.n + v] = val;
  }
}

struct MsStats {
  u64 newbits = 0, comp = 0, active = 0, active_out = 0, done_in = 0, scanned = 0;
  __device__ __forceinline__ void flush(MsCtr *sh) {
    MsCtr *c = sh + (blockIdx.x % NSH);
    u64 v[6] = {wave_sum_u64(newbits), wave_sum_u64(comp), wave_sum_u64(active), wave_sum_u64(active_out),
                wave_sum_u64(done_in), wave_sum_u64(scanned)};
    if (lane() == 0) {
      u64 *f = reinterpret_cast<u64 *>(c);
      for (int j = 0; j < 6; ++j)
        if (v[j]) atomicAdd(f + j, v[j]);
    }
  }
};

__device__ __forceinline__ void ms_clear_dead(const MsArgs &a) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthr = gridDim.x * blockDim.x;
  for (int i = tid; i < a.n; i += nthr) a.dead[i] = 0ull;
}

// Records the discovery of `nw` lanes at v (owner thread): vis, depths, stats.
__device__ __forceinline__ void ms_discover(const MsArgs &a, int v, u64 vis_old, u64 nw, MsStats &st) {
  const u64 vnew = vis_old | nw;
  a.vis[v] = vnew;
  ms_write_levels(a, v, nw, a.k + 1);
  const int c = __popcll(nw);
  const int od = a.rp[v + 1] - a.rp[v];
  st.newbits += (u64)c;
  st.comp += (u64)c * (u64)od;
  st.active += 1;
  st.active_out += (u64)od;
  if ((vnew & a.full) == a.full) st.done_in += (u64)(a.cp[v + 1] - a.cp[v]);
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(BLOCK) void k_ms_init(MsArgs a, u64 *f0, u64 *f1, u64 *f2) {
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
    a.vis[v] = 0ull;
    f0[v] = 0ull;
    f1[v] = 0ull;
    f2[v] = 0ull;
  }
}

// One thread per lane: sets the source bit and depth 0 (duplicates OR).
__global__ void k_ms_sources(MsArgs a, const int *src, u64 *f0) {
  const int l = threadIdx.x;
  if (l < a.L) {
    const int s = src[l];
    atomicOr(a.vis + s, 1ull << l);
    atomicOr(f0 + s, 1ull << l);
    a.levels[(size_t)l * a.n + s] = 0;
  }
}

// ------------------------------------------------------------------ pull
__global__ __launch_bounds__(BLOCK) void k_ms_pull(MsArgs a) {
  ms_clear_dead(a);
  MsStats st;
  const int wv = threadIdx.x / WAVE;
  const int nwords = (a.n + WAVE - 1) / WAVE;
  for (int w = blockIdx.x * (BLOCK / WAVE) + wv; w < nwords; w += gridDim.x * (BLOCK / WAVE)) {
    const int v = w * WAVE + lane();
    u64 vw = 0, need = 0, acc = 0;
    int b = 0, e = 0;
    bool pending = false;
    if (v < a.n) {
      vw = a.vis[v];
      need = a.full & ~vw;
      if (need) {
        b = a.cp[v];
        e = a.cp[v + 1];
        const int d = e - b;
        int u[MS_T];
#pragma unroll
        for (int t = 0; t < MS_T; ++t) u[t] = (t < d) ? a.cx[b + t] : -1;
#pragma unroll
        for (int t = 0; t < MS_T; ++t) acc |= (u[t] >= 0) ? a.front[u[t]] : 0ull;
        st.scanned += (u64)min(d, MS_T);
        pending = d > MS_T && (acc & need) != need;
        b += MS_T;
      }
    }
    u64 pm = __ballot(pending);
    while (pm) {
      const int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      const int vb = __shfl(b, l), ve = __shfl(e, l);
      const u64 ln = __shfl(need, l);
      u64 wacc = __shfl(acc, l);
      for (int base = vb; base < ve; base += WAVE) {
        const int j = base + lane();
        u64 f = (j < ve) ? a.front[a.cx[j]] : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o);
        wacc |= f;
        if (lane() == l) st.scanned += (u64)min(WAVE, ve - base);
        if ((wacc & ln) == ln) break;
      }
      if (lane() == l) acc = wacc;
    }
    if (v < a.n) {
      const u64 nw = acc & need;
      a.next[v] = nw;
      if (nw) ms_discover(a, v, vw, nw, st);
    }
  }
  st.flush(a.sh);
}

// ------------------------------------------------------------------ push
__global__ __launch_bounds__(BLOCK) void k_ms_push(MsArgs a) {
  ms_clear_dead(a);
  MsStats st;
  const int wv = threadIdx.x / WAVE;
  const int nwords = (a.n + WAVE - 1) / WAVE;
  for (int w = blockIdx.x * (BLOCK / WAVE) + wv; w < nwords; w += gridDim.x * (BLOCK / WAVE)) {
    const int u = w * WAVE + lane();
    const u64 fu = (u < a.n) ? a.front[u] : 0ull;
    const u64 am = __ballot(fu != 0ull);
    if (!am) continue;
    int b = 0, e = 0;
    bool pending = false;
    if (fu) {
      b = a.rp[u];
      e = a.rp[u + 1];
      const int d = e - b;
#pragma unroll
      for (int t = 0; t < MS_T; ++t)
        if (t < d) {
          const int v = a.ci[b + t];
          const u64 m = fu & ~a.vis[v];
          if (m) atomicOr(a.next + v, m);
        }
      st.scanned += (u64)min(d, MS_T);
      pending = d > MS_T;
      b += MS_T;
    }
    u64 pm = __ballot(pending);
    while (pm) {
      const int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      const int vb = __shfl(b, l), ve = __shfl(e, l);
      const u64 lf = __shfl(fu, l);
      for (int j = vb + lane(); j < ve; j += WAVE) {
        const int v = a.ci[j];
        const u64 m = lf & ~a.vis[v];
        if (m) atomicOr(a.next + v, m);
      }
      if (lane() == l) st.scanned += (u64)(ve - vb);
    }
  }
  st.flush(a.sh);
}

// Owner-computes update after a push: F_{k+1}[v] = next[v] (already masked).
__global__ __launch_bounds__(BLOCK) void k_ms_push_update(MsArgs a) {
  MsStats st;
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
    const u64 nw = a.next[v];
    if (nw) ms_discover(a, v, a.vis[v], nw, st);
  }
  st.flush(a.sh);
}

// Depth -1 for every lane that never reached v.
__global__ __launch_bounds__(BLOCK) void k_ms_final(MsArgs a) {
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK)
    ms_write_levels(a, v, a.full & ~a.vis[v], -1);
}

__global__ __launch_bounds__(NSH) void k_ms_finish(MsCtr *sh, MsCtr *tot) {
  __shared__ u64 s_red[6][NSH / WAVE];
  const int t = threadIdx.x;
  const u64 *f = reinterpret_cast<const u64 *>(sh + t);
  for (int j = 0; j < 6; ++j) {
    u64 r = wave_sum_u64(f[j]);
    if (lane() == 0) s_red[j][t / WAVE] = r;
  }
  __syncthreads();
  if (t < 6) {
    u64 r = 0;
    for (int i = 0; i < NSH / WAVE; ++i) r += s_red[t][i];
    reinterpret_cast<u64 *>(tot)[t] = r;
  }
}

__global__ void k_ms_zero(MsCtr *sh) {
  u64 *f = reinterpret_cast<u64 *>(sh);
  for (int i = threadIdx.x; i < NSH * 8; i += blockDim.x) f[i] = 0ull;
}

// Out-degree of each lane's source (for the F_0 counts and the component
// edge total).
__global__ void k_ms_src_deg(const int *rp, const int *src, int L, int *deg) {
  const int l = threadIdx.x;
  if (l < L) deg[l] = rp[src[l] + 1] - rp[src[l]];
}

}  // namespace bfs

using namespace bfs;

extern "C" int bfs_multi(const bfs_graph *g, const int32_t *sources, int32_t k, int32_t *levels,
                         const bfs_options *opt, bfs_stats *st, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!g || g->n <= 0 || !g->row_ptr || (!g->col_idx && g->nnz > 0) || !sources || !levels || k < 1) {
    set_error("bfs_multi: invalid argument (null pointer, n <= 0 or k < 1)");
    return BFS_EINVAL;
  }
  if (!g->csc_ptr || !g->csc_idx) {
    set_error("bfs_multi needs CSC arrays (pass the CSR again for a symmetric graph)");
    return BFS_ENOTSUP;
  }
  for (int i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) {
      set_error("bfs_multi: source %d (index %d) out of range", sources[i], i);
      return BFS_EINVAL;
    }
  const int n = g->n;
  const int mode = opt ? opt->variant : BFS_AUTO_HEURISTIC;
  const size_t need = workspace_bytes_multi(n);
  void *wsp = opt ? opt->workspace : nullptr;
  int rc;
  if (wsp) {
    if (opt->workspace_bytes < need) {
      set_error("workspace has %zu bytes, needs %zu", opt->workspace_bytes, need);
      return BFS_EWORKSPACE;
    }
  } else {
    rc = cached_workspace(need, &wsp);
    if (rc) return rc;
  }
  char *p = (char *)wsp;
  const size_t vb = ((size_t)n * 8 + 255) & ~(size_t)255;
  u64 *fr[3] = {(u64 *)p, (u64 *)(p + vb), (u64 *)(p + 2 * vb)};
  u64 *vis = (u64 *)(p + 3 * vb);
  MsCtr *sh = (MsCtr *)(p + 4 * vb);       // NSH shards
  MsCtr *tot = sh + NSH;                   // reduced totals
  int *src_dev = (int *)(tot + 1);         // [64] sources of the group, [64] their degrees
  HostCtx &hc = host_ctx();
  const int grid_v = std::min(4096, (n + BLOCK - 1) / BLOCK);
  const int grid_w = std::min(4096, ((n + WAVE - 1) / WAVE + 3) / 4);
  long long reached = 0, comp = 0;
  int max_levels = 0, syncs = 0;
  BFS_HIP(hipEventRecord(hc.ev[0], s));
  for (int g0 = 0; g0 < k; g0 += 64) {
    const int L = std::min(64, k - g0);
    MsArgs a;
    a.n = n;
    a.k = 0;
    a.L = L;
    a.full = (L == 64) ? ~0ull : ((1ull << L) - 1);
    a.rp = g->row_ptr;
    a.ci = g->col_idx;
    a.cp = g->csc_ptr;
    a.cx = g->csc_idx;
    a.vis = vis;
    a.levels = levels + (size_t)g0 * n;
    a.sh = sh;
    hipLaunchKernelGGL(k_ms_init, dim3(grid_v), dim3(BLOCK), 0, s, a, fr[0], fr[1], fr[2]);
    BFS_HIP(hipMemcpyAsync(src_dev, sources + g0, L * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ms_sources, dim3(1), dim3(64), 0, s, a, (const int *)src_dev, fr[0]);
    // counts of F_0 for the direction rule: distinct source vertices and their degrees
    hipLaunchKernelGGL(k_ms_src_deg, dim3(1), dim3(64), 0, s, g->row_ptr, (const int *)src_dev, L, src_dev + 64);
    BFS_HIP(hipGetLastError());
    int *deg_host = reinterpret_cast<int *>(hc.pinned_u64);
    BFS_HIP(hipMemcpyAsync(deg_host, src_dev + 64, L * sizeof(int), hipMemcpyDeviceToHost, s));
    BFS_HIP(hipStreamSynchronize(s));
    long long nf = 0, ef = 0, src_comp = 0;
    {
      std::vector<std::pair<int, int>> sd;
      for (int i = 0; i < L; ++i) {
        sd.push_back({sources[g0 + i], deg_host[i]});
        src_comp += deg_host[i];
      }
      std::sort(sd.begin(), sd.end());
      for (size_t i = 0; i < sd.size(); ++i)
        if (i == 0 || sd[i].first != sd[i - 1].first) {
          ++nf;
          ef += sd[i].second;
        }
    }
    long long eu = g->nnz;  // in-edges of vertices still missing some lane
    reached += L;
    HeuristicState hs;
    int lev = 0;
    for (;;) {
      int dir;
      if (mode == BFS_V_PUSH_Q_THREAD || mode == BFS_V_PUSH_Q_BLOCK || mode == BFS_V_PUSH_Q_MERGE)
        dir = 0;
      else if (mode == BFS_V_PULL_B)
        dir = 1;
      else {
        hs.step(n, nf, ef, eu);
        dir = hs.dir;
      }
      a.k = lev;
      a.front = fr[lev % 3];
      a.next = fr[(lev + 1) % 3];
      a.dead = fr[(lev + 2) % 3];
      hipLaunchKernelGGL(k_ms_zero, dim3(1), dim3(BLOCK), 0, s, sh);
      if (dir == 1) {
        hipLaunchKernelGGL(k_ms_pull, dim3(grid_w), dim3(BLOCK), 0, s, a);
      } else {
        hipLaunchKernelGGL(k_ms_push, dim3(grid_w), dim3(BLOCK), 0, s, a);
        hipLaunchKernelGGL(k_ms_push_update, dim3(grid_v), dim3(BLOCK), 0, s, a);
      }
      hipLaunchKernelGGL(k_ms_finish, dim3(1), dim3(NSH), 0, s, sh, tot);
      BFS_HIP(hipGetLastError());
      BFS_HIP(hipMemcpyAsync(hc.pinned, tot, sizeof(MsCtr), hipMemcpyDeviceToHost, s));
      BFS_HIP(hipStreamSynchronize(s));
      ++syncs;
      MsCtr c;
      memcpy(&c, hc.pinned, sizeof(c));
      ++lev;
      if (c.newbits == 0) break;
      reached += (long long)c.newbits;
      comp += (long long)c.comp_edges;
      nf = (long long)c.active;
      ef = (long long)c.active_out;
      eu -= (long long)c.done_in;
      if (lev > n + 1) {
        set_error("bfs_multi: level loop did not converge");
        return BFS_ELEVELCAP;
      }
    }
    comp += src_comp;  // each lane's source belongs to its component
    hipLaunchKernelGGL(k_ms_final, dim3(grid_v), dim3(BLOCK), 0, s, a);
    BFS_HIP(hipGetLastError());
    max_levels = std::max(max_levels, lev);
  }
  BFS_HIP(hipEventRecord(hc.ev[1], s));
  BFS_HIP(hipEventSynchronize(hc.ev[1]));
  if (st) {
    float ms = 0.f;
    BFS_HIP(hipEventElapsedTime(&ms, hc.ev[0], hc.ev[1]));
    st->num_levels = max_levels;
    st->reached = reached;
    st->component_edges = comp;
    st->elapsed_ms = ms;
    st->host_syncs = syncs;
  }
  return BFS_OK;
}
