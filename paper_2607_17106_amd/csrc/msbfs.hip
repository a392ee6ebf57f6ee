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
// reduction, stopping once every lane the vertex lacks has been found.  An
// in-neighbour's frontier word is gathered only when its bit is set in the
// any-lane frontier bitmap (n/8 bytes, cache resident), so edges from
// vertices outside the frontier cost a column id and one bit.
// Push (top-down, CSR): frontier vertices OR their frontier word, masked by
// the target's (read-only) visited word, into the target's next word with
// atomicOr; an owner-computes pass then applies the update.
//
// Depths are not written during the levels.  Each discovery ORs the new lane
// bits into bit planes of the relative depth r = k + 1 - base (bit l of plane
// b is bit b of lane l's r); one output pass then writes every row of the
// [lanes][n] depth array once, in whole coalesced lines.  When r would need
// more than MS_PLANES planes, a flush pass writes the lanes found so far,
// marks them, and a new window starts at base = k.
#include <string.h>
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "selector.hpp"

namespace bfs {

constexpr int MS_T = 4;
constexpr long long MS_ALPHA = 4;  // bottom-up when frontier out-edges exceed 1/4 of eu
constexpr int MS_PLANES = 8;       // relative depths 0..255 per window

struct MsCtr {  // one 64-byte line per shard
  u64 newbits;     // (lane, vertex) pairs discovered
  u64 comp_edges;  // sum over discoveries of outdeg(v) (per lane)
  u64 active;      // vertices with at least one new lane (next frontier size)
  u64 active_out;  // their out-edges
  u64 done_in;     // in-edges of vertices whose last lane was found
  u64 scanned;     // edges examined
  u64 unvis;       // vertices still missing some lane when the step started
  u64 hits;        // examined edges whose source is in the frontier (words gathered)
};
static_assert(sizeof(MsCtr) == 64, "MsCtr is one line");
constexpr int MS_NCTR = 8;

struct MsArgs {
  int n, k, L;          // vertices, level, lanes in this group
  int rel;              // relative depth of this step's discoveries (k + 1 - base)
  u64 full;             // mask of the L lanes
  const int *rp, *ci, *cp, *cx;
  const u64 *front;     // F_k words
  const u64 *fbits;     // any-lane bitmap of F_k: bit v%64 of word v/64
  u64 *next;            // F_{k+1} words
  u64 *nbits;           // any-lane bitmap of F_{k+1}, every word written by the step
  u64 *dead;            // buffer to clear for F_{k+2}
  u64 *vis;
  u64 *planes;          // plane b at planes + b * n
  u64 *flushed;         // lanes whose depths a flush pass has written
  int *levels;          // row l at levels + l * n
  int base, np, nflush; // output passes: window base, planes in use, flushes so far
  MsCtr *sh;            // NSH shards of this level's counters
};

struct MsCarve {
  u64 *fr[3], *vis, *flushed, *planes, *fb[2];
  MsCtr *sh, *tot;
  int *src;             // [64] sources of the group, [64] their degrees
  size_t bytes;
};

static MsCarve ms_carve(uintptr_t p, int n) {
  const auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t vb = al((size_t)n * 8), bb = al(((size_t)n + 63) / 64 * 8);
  MsCarve c;
  size_t off = 0;
  for (int i = 0; i < 3; ++i, off += vb) c.fr[i] = reinterpret_cast<u64 *>(p + off);
  c.vis = reinterpret_cast<u64 *>(p + off);
  off += vb;
  c.flushed = reinterpret_cast<u64 *>(p + off);
  off += vb;
  c.planes = reinterpret_cast<u64 *>(p + off);
  off += al((size_t)MS_PLANES * n * 8);
  for (int i = 0; i < 2; ++i, off += bb) c.fb[i] = reinterpret_cast<u64 *>(p + off);
  c.sh = reinterpret_cast<MsCtr *>(p + off);
  c.tot = c.sh + NSH;
  off += (size_t)(NSH + 1) * sizeof(MsCtr);
  c.src = reinterpret_cast<int *>(p + off);
  off += 512;
  c.bytes = off;
  return c;
}

size_t workspace_bytes_multi(int n) { return ms_carve(0, n).bytes; }

__device__ __forceinline__ bool in_front(const u64 *fb, int u) { return (fb[u >> 6] >> (u & 63)) & 1ull; }

struct MsStats {
  u64 c[MS_NCTR] = {0, 0, 0, 0, 0, 0, 0, 0};
  __device__ __forceinline__ void flush(MsCtr *sh) {
    u64 *f = reinterpret_cast<u64 *>(sh + (blockIdx.x % NSH));
#pragma unroll
    for (int j = 0; j < MS_NCTR; ++j) {
      const u64 r = wave_sum_u64(c[j]);
      if (lane() == 0 && r) atomicAdd(f + j, r);
    }
  }
};
enum { C_NEW, C_COMP, C_ACTIVE, C_ACTOUT, C_DONEIN, C_SCAN, C_UNVIS, C_HITS };

__device__ __forceinline__ void ms_clear_dead(const MsArgs &a) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthr = gridDim.x * blockDim.x;
  for (int i = tid; i < a.n; i += nthr) a.dead[i] = 0ull;
}

// Records the discovery of `nw` lanes at v (owner thread, so the plane
// updates are plain read-modify-writes): vis, depth planes, stats.
__device__ __forceinline__ void ms_discover(const MsArgs &a, int v, u64 vis_old, u64 nw, MsStats &st) {
  const u64 vnew = vis_old | nw;
  a.vis[v] = vnew;
  for (int r = a.rel, b = 0; r; r >>= 1, ++b)
    if (r & 1) a.planes[(size_t)b * a.n + v] |= nw;
  const int c = __popcll(nw);
  const int od = a.rp[v + 1] - a.rp[v];
  st.c[C_NEW] += (u64)c;
  st.c[C_COMP] += (u64)c * (u64)od;
  st.c[C_ACTIVE] += 1;
  st.c[C_ACTOUT] += (u64)od;
  if ((vnew & a.full) == a.full) st.c[C_DONEIN] += (u64)(a.cp[v + 1] - a.cp[v]);
}

// Writes the depth of every lane of v not in `skip`: a.base + r for visited
// lanes (r read from the NP planes in use), -1 for the others.  Called by
// whole waves holding 64 consecutive vertices, so each of the L row stores
// covers 64 consecutive ints; lanes with valid = false store nothing.  The
// planes are split into 32-bit halves so one bit-field extract per plane
// gives a lane's bit.
template <int NP>
__device__ __forceinline__ void ms_store_depths(const MsArgs &a, int v, bool valid, u64 vw, u64 skip) {
  uint32_t pl[2][NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const u64 w = valid ? a.planes[(size_t)b * a.n + v] : 0ull;
    pl[0][b] = (uint32_t)w;
    pl[1][b] = (uint32_t)(w >> 32);
  }
  const u64 store = valid ? ~skip : 0ull;
  int *out = a.levels + v;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t vis_h = (uint32_t)(vw >> (32 * h)), st_h = (uint32_t)(store >> (32 * h));
    const int lend = min(a.L - 32 * h, 32);
    for (int l = 0; l < lend; ++l, out += a.n) {
      int r = 0;
#pragma unroll
      for (int b = 0; b < NP; ++b) r |= (int)((pl[h][b] >> l) & 1u) << b;
      if ((st_h >> l) & 1u) *out = ((vis_h >> l) & 1u) ? a.base + r : -1;
    }
  }
}

template <int NP>
__device__ __forceinline__ void ms_out_body(const MsArgs &a, int flush) {
  for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {  // uniform per wave
    const int v = base + threadIdx.x;
    const bool valid = v < a.n;
    const u64 vw = valid ? a.vis[v] & a.full : 0ull;
    const u64 fl = (valid && a.nflush) ? a.flushed[v] : 0ull;
    if (flush) {
      ms_store_depths<NP>(a, v, valid, vw, ~(vw & ~fl));
      if (valid) a.flushed[v] = vw;
    } else {
      ms_store_depths<NP>(a, v, valid, vw, fl);
    }
  }
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(BLOCK) void k_ms_init(MsArgs a, u64 *f0, u64 *f1, u64 *b0) {
  const int nw = (a.n + 63) / 64;
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
    a.vis[v] = 0ull;
    f0[v] = 0ull;
    f1[v] = 0ull;
    if (v < nw) b0[v] = 0ull;
  }
}

// One thread per lane: sets the source bit (duplicates OR); depth 0 is
// relative depth 0, which the zeroed planes already hold.
__global__ void k_ms_sources(MsArgs a, const int *src, u64 *f0, u64 *b0) {
  const int l = threadIdx.x;
  if (l < a.L) {
    const int s = src[l];
    atomicOr(a.vis + s, 1ull << l);
    atomicOr(f0 + s, 1ull << l);
    atomicOr(b0 + (s >> 6), 1ull << (s & 63));
  }
}

__global__ __launch_bounds__(BLOCK) void k_ms_fill(u64 *p, int n) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) p[i] = 0ull;
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
        st.c[C_UNVIS] += 1;
        b = a.cp[v];
        e = a.cp[v + 1];
        const int d = e - b;
        int u[MS_T];
#pragma unroll
        for (int t = 0; t < MS_T; ++t) u[t] = (t < d) ? a.cx[b + t] : -1;
        bool hit[MS_T];
#pragma unroll
        for (int t = 0; t < MS_T; ++t) hit[t] = u[t] >= 0 && in_front(a.fbits, u[t]);
#pragma unroll
        for (int t = 0; t < MS_T; ++t)
          if (hit[t]) {
            acc |= a.front[u[t]];
            st.c[C_HITS] += 1;
          }
        st.c[C_SCAN] += (u64)min(d, MS_T);
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
        u64 f = 0ull;
        if (j < ve) {
          const int u = a.cx[j];
          if (in_front(a.fbits, u)) {
            f = a.front[u];
            st.c[C_HITS] += 1;
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o);
        wacc |= f;
        if (lane() == l) st.c[C_SCAN] += (u64)min(WAVE, ve - base);
        if ((wacc & ln) == ln) break;
      }
      if (lane() == l) acc = wacc;
    }
    u64 nw = 0ull;
    if (v < a.n) {
      nw = acc & need;
      a.next[v] = nw;
      if (nw) ms_discover(a, v, vw, nw, st);
    }
    const u64 nb = __ballot(nw != 0ull);
    if (lane() == 0) a.nbits[w] = nb;
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
    const u64 wb = a.fbits[w];
    if (!wb) continue;  // no frontier vertex among these 64
    const int u = w * WAVE + lane();
    const u64 fu = ((wb >> lane()) & 1ull) ? a.front[u] : 0ull;
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
      st.c[C_SCAN] += (u64)min(d, MS_T);
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
      if (lane() == l) st.c[C_SCAN] += (u64)(ve - vb);
    }
  }
  st.flush(a.sh);
}

// Owner-computes update after a push: F_{k+1}[v] = next[v] (already masked).
__global__ __launch_bounds__(BLOCK) void k_ms_push_update(MsArgs a) {
  MsStats st;
  for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {  // uniform per wave
    const int v = base + threadIdx.x;
    const u64 nw = v < a.n ? a.next[v] : 0ull;
    if (nw) ms_discover(a, v, a.vis[v], nw, st);
    const u64 nb = __ballot(nw != 0ull);
    const int w = (base + (int)(threadIdx.x & ~(WAVE - 1))) / WAVE;
    if (lane() == 0 && w * WAVE < a.n) a.nbits[w] = nb;
  }
  st.flush(a.sh);
}

// Output pass.  flush = 0: the final pass, every lane not yet written (depth
// from the planes, or -1).  flush = 1: the lanes visited since the last
// flush, which are then marked in `flushed`.
__global__ __launch_bounds__(BLOCK) void k_ms_out(MsArgs a, int flush) {
  switch (a.np) {
    case 0:
    case 1: ms_out_body<1>(a, flush); break;
    case 2: ms_out_body<2>(a, flush); break;
    case 3: ms_out_body<3>(a, flush); break;
    case 4: ms_out_body<4>(a, flush); break;
    case 5: ms_out_body<5>(a, flush); break;
    case 6: ms_out_body<6>(a, flush); break;
    case 7: ms_out_body<7>(a, flush); break;
    default: ms_out_body<MS_PLANES>(a, flush); break;
  }
}

__global__ __launch_bounds__(NSH) void k_ms_finish(MsCtr *sh, MsCtr *tot) {
  __shared__ u64 s_red[MS_NCTR][NSH / WAVE];
  const int t = threadIdx.x;
  const u64 *f = reinterpret_cast<const u64 *>(sh + t);
  for (int j = 0; j < MS_NCTR; ++j) {
    u64 r = wave_sum_u64(f[j]);
    if (lane() == 0) s_red[j][t / WAVE] = r;
  }
  __syncthreads();
  if (t < MS_NCTR) {
    u64 r = 0;
    for (int i = 0; i < NSH / WAVE; ++i) r += s_red[t][i];
    reinterpret_cast<u64 *>(tot)[t] = r;
  }
}

__global__ void k_ms_zero(MsCtr *sh) {
  u64 *f = reinterpret_cast<u64 *>(sh);
  for (int i = threadIdx.x; i < NSH * MS_NCTR; i += blockDim.x) f[i] = 0ull;
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
  const MsCarve W = ms_carve(reinterpret_cast<uintptr_t>(wsp), n);
  u64 *const *fr = W.fr;
  MsCtr *sh = W.sh, *tot = W.tot;
  int *src_dev = W.src;
  HostCtx &hc = host_ctx();
  const int grid_v = std::min(4096, (n + BLOCK - 1) / BLOCK);
  const int grid_w = std::min(4096, ((n + WAVE - 1) / WAVE + 3) / 4);
  long long reached = 0, comp = 0;
  int max_levels = 0, syncs = 0;
  const int flags = opt ? opt->flags : 0;
  const bool rec = st && (flags & (BFS_F_LEVEL_STATS | BFS_F_LEVEL_TIMING)) && st->level_capacity > 0;
  const bool timing = rec && (flags & BFS_F_LEVEL_TIMING);
  int recorded = 0;
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
    a.vis = W.vis;
    a.planes = W.planes;
    a.flushed = W.flushed;
    a.levels = levels + (size_t)g0 * n;
    a.sh = sh;
    a.base = 0;
    a.np = 0;
    a.nflush = 0;
    hipLaunchKernelGGL(k_ms_init, dim3(grid_v), dim3(BLOCK), 0, s, a, fr[0], fr[1], W.fb[0]);
    BFS_HIP(hipMemcpyAsync(src_dev, sources + g0, L * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ms_sources, dim3(1), dim3(64), 0, s, a, (const int *)src_dev, fr[0], W.fb[0]);
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
    int msdir = 0;
    long long prev_nf = -1;
    int lev = 0;
    for (;;) {
      int dir;
      if (mode == BFS_V_PUSH_Q_THREAD || mode == BFS_V_PUSH_Q_BLOCK || mode == BFS_V_PUSH_Q_MERGE)
        dir = 0;
      else if (mode == BFS_V_PULL_B)
        dir = 1;
      else {
        // Direction rule for bit-packed lanes: a bottom-up step exits early
        // only once every lane a vertex misses is found, so it costs close to
        // all in-edges of the vertices still missing a lane (eu); top-down
        // costs the frontier's out-edges (ef).  Bottom-up when
        // ef > eu / MS_ALPHA; back to top-down under Beamer's beta test.
        if (msdir == 0) {
          if (ef * MS_ALPHA > eu) msdir = 1;
        } else if (nf * HeuristicState::kBeta < (long long)n && prev_nf >= 0 && nf < prev_nf) {
          msdir = 0;
        }
        prev_nf = nf;
        dir = msdir;
      }
      // relative depth of this step's discoveries; a full window is written out first
      if (lev + 1 - a.base >= (1 << MS_PLANES)) {
        hipLaunchKernelGGL(k_ms_out, dim3(grid_v), dim3(BLOCK), 0, s, a, 1);
        ++a.nflush;
        a.base = lev;
        a.np = 0;
      }
      a.rel = lev + 1 - a.base;
      while ((a.rel >> a.np) != 0) {  // zero each plane on its first use in the window
        hipLaunchKernelGGL(k_ms_fill, dim3(grid_v), dim3(BLOCK), 0, s, a.planes + (size_t)a.np * n, n);
        ++a.np;
      }
      a.k = lev;
      a.front = fr[lev % 3];
      a.next = fr[(lev + 1) % 3];
      a.dead = fr[(lev + 2) % 3];
      a.fbits = W.fb[lev & 1];
      a.nbits = W.fb[(lev + 1) & 1];
      hipLaunchKernelGGL(k_ms_zero, dim3(1), dim3(BLOCK), 0, s, sh);
      if (timing) BFS_HIP(hipEventRecord(hc.ev[2], s));
      if (dir == 1) {
        hipLaunchKernelGGL(k_ms_pull, dim3(grid_w), dim3(BLOCK), 0, s, a);
      } else {
        hipLaunchKernelGGL(k_ms_push, dim3(grid_w), dim3(BLOCK), 0, s, a);
        hipLaunchKernelGGL(k_ms_push_update, dim3(grid_v), dim3(BLOCK), 0, s, a);
      }
      if (timing) BFS_HIP(hipEventRecord(hc.ev[3], s));
      hipLaunchKernelGGL(k_ms_finish, dim3(1), dim3(NSH), 0, s, sh, tot);
      BFS_HIP(hipGetLastError());
      BFS_HIP(hipMemcpyAsync(hc.pinned, tot, sizeof(MsCtr), hipMemcpyDeviceToHost, s));
      BFS_HIP(hipStreamSynchronize(s));
      ++syncs;
      MsCtr c;
      memcpy(&c, hc.pinned, sizeof(c));
      if (rec && recorded < st->level_capacity) {
        // entry: one level of one group; variant 6 = bottom-up, 0 = top-down
        const int r = recorded++;
        if (st->level_variant) st->level_variant[r] = dir == 1 ? BFS_V_PULL_B : BFS_V_PUSH_Q_THREAD;
        if (st->level_frontier) st->level_frontier[r] = nf;
        if (st->level_frontier_edges) st->level_frontier_edges[r] = ef;
        if (st->level_unvisited) st->level_unvisited[r] = (long long)c.unvis;
        if (st->level_unvisited_edges) st->level_unvisited_edges[r] = eu;
        if (st->level_scanned) st->level_scanned[r] = (long long)c.scanned;
        if (st->level_next) st->level_next[r] = (long long)c.newbits;
        if (st->level_frontier_ld) st->level_frontier_ld[r] = (long long)c.active;
        if (st->level_frontier_ld2) st->level_frontier_ld2[r] = (long long)c.hits;
        if (st->level_ms) {
          float ms = 0.f;
          if (timing) BFS_HIP(hipEventElapsedTime(&ms, hc.ev[2], hc.ev[3]));
          st->level_ms[r] = ms;
        }
      }
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
    hipLaunchKernelGGL(k_ms_out, dim3(grid_v), dim3(BLOCK), 0, s, a, 0);
    BFS_HIP(hipGetLastError());
    max_levels = std::max(max_levels, lev);
  }
  BFS_HIP(hipEventRecord(hc.ev[1], s));
  BFS_HIP(hipEventSynchronize(hc.ev[1]));
  if (st) {
    float ms = 0.f;
    BFS_HIP(hipEventElapsedTime(&ms, hc.ev[0], hc.ev[1]));
    st->num_levels = rec ? recorded : max_levels;
    st->reached = reached;
    st->component_edges = comp;
    st->elapsed_ms = ms;
    st->host_syncs = syncs;
  }
  return BFS_OK;
}
