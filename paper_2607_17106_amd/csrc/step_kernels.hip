// Level-step kernels of single-source BFS for gfx950 (wave64).
//
// One level expands F_k into F_{k+1} (Cascade 1, Eq. advance) and merges it
// into the visited set P (Eq. update).  Layout: visited P and frontier
// bitmaps are u64 words (bit v&63 of word v>>6); frontier queues are int32
// vertex lists split into NSH segments (see common.hpp); depths/parents are
// int32 per vertex.
//
// Push (top-down) kernels walk out-edges of F_k (loop order s -> d, Sec.
// "The Einsum-Enabled Design Space", B.1) and claim each unvisited d:
//   ATOM = true : one atomicOr on d's visited word decides the single winner,
//                 which writes depth/parent and appends d (Table 3, variants
//                 1-3 and 10).
//   ATOM = false: the visited bitmap is a read-only mask for the whole step;
//                 every lane that sees d unvisited stores depth k+1 (the same
//                 value, so the race is benign) and some parent; a separate
//                 owner-computes pass then derives F_{k+1} from the depths and
//                 updates P (Table 3, variants 12, 21, 24: mask, no atomics,
//                 P_{i+1} = P_i OR F_{i+1}).
// Pull (bottom-up) walks in-edges of unvisited vertices and stops at the first
// frontier member (Sec. "From Push to Pull BFS", loop order d -> s).
//
// Load balance over the frontier's edge space (Sec. "Load Balancing
// Strategies"; Table 3, variants 1-3):
//   thread : one lane per frontier vertex walks its whole row.
//   block  : partition the queue into chunks of 256 vertices, flatten each
//            chunk's (vertex, edge) space with a workgroup scan, split it
//            evenly over the 256 lanes; vertices above the hub threshold are
//            deferred to a second kernel that splits them across the grid.
//   merge  : flatten the whole frontier's edge space with a device-wide
//            degree scan and cut it into equal tiles; each tile finds its
//            first vertex with a 64-ary wave search (merge-path partition).
//
// No kernel takes a device-scope atomic on a single hot address: counters
// and queue reservations go to the workgroup's shard (common.hpp).
#include <algorithm>

#include "common.hpp"

namespace bfs {

// ------------------------------------------------------------------ reset
// One wave per bitmap word.  Vertices without in-edges can never be
// discovered; their visited bits are set up front so no step searches them
// (their depth stays -1).  That needs in-degrees, i.e. CSC arrays (or a
// symmetric CSR passed as its own CSC).
__global__ __launch_bounds__(BLOCK) void k_reset(StepArgs a, int src, RingSlot *ring) {
  const int wv = threadIdx.x / WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  for (int w = gw; w < a.W; w += nw) {
    const int v = w * WAVE + lane();
    bool dead = false;
    if (v < a.n) {
      a.levels[v] = (v == src) ? 0 : -1;
      if (a.parents) a.parents[v] = (v == src) ? src : -1;
      dead = a.cp && (a.cp[v + 1] == a.cp[v]) && v != src;
    }
    const u64 dm = __ballot(dead || v >= a.n);
    if (lane() == 0) {
      const u64 sb = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
      a.vis[w] = sb | dm;
      const_cast<u64 *>(a.fb_cur)[w] = sb;
      a.fb_next[w] = 0;
      a.fb_dead[w] = 0;
    }
  }
  // zero every shard of every slot
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthr = gridDim.x * blockDim.x;
  const int per = (int)(sizeof(RingSlot) / sizeof(u32));
  u32 *z = reinterpret_cast<u32 *>(ring);
  for (int i = tid; i < RING * per; i += nthr) z[i] = 0u;
  if (tid == 0) const_cast<int *>(a.q_cur)[0] = src;
}

// Writes F_0 = {src} into slot 0's total and segment offsets (after k_reset
// has zeroed the ring): the source sits alone in segment 0.
__global__ void k_reset_f0(StepArgs a, int src, RingSlot *slot0) {
  const int t = threadIdx.x;
  if (t < NSH + 2) slot0->seg[t] = (t == 0) ? 0 : 1;
  if (t == 0) {
    LevelCtr &c = slot0->tot;
    int d = a.rp[src + 1] - a.rp[src];
    int di = a.cp ? a.cp[src + 1] - a.cp[src] : d;
    int l = ilog2p1(d);
    c.count = 1;
    c.edges = (u64)d;
    c.in_edges = (u64)di;
    c.ld = (u64)l;
    c.ld2 = (u64)(l * l);
    c.decision = -1;
  }
}

// ------------------------------------------------------------- finish
// Reduces the NSH shards of one slot into its total and the queue segment
// offsets.  One workgroup of NSH threads.
__global__ __launch_bounds__(NSH) void k_finish(RingSlot *slot, int qcap) {
  __shared__ int s_w[NSH / WAVE];
  __shared__ u64 s_red[5][NSH / WAVE];
  const int t = threadIdx.x;
  const LevelCtr &c = slot->sh[t];
  const int cnt = (int)min(c.count, (u32)qcap);
  const int w = t / WAVE;
  const int incl = wave_incl_scan(cnt);
  if (lane() == WAVE - 1) s_w[w] = incl;
  u64 v[5] = {c.edges, c.in_edges, c.ld, c.ld2, c.scanned};
  for (int j = 0; j < 5; ++j) {
    u64 r = wave_sum_u64(v[j]);
    if (lane() == 0) s_red[j][w] = r;
  }
  __syncthreads();
  int off = 0, total = 0;
  for (int i = 0; i < NSH / WAVE; ++i) {
    off += (i < w) ? s_w[i] : 0;
    total += s_w[i];
  }
  slot->seg[t] = off + incl - cnt;
  if (t == 0) {
    const int ovf = (int)slot->sh[NSH].count;
    slot->seg[NSH] = total;
    slot->seg[NSH + 1] = total + ovf;
    LevelCtr &o = slot->tot;
    u64 r[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < 5; ++j)
      for (int i = 0; i < NSH / WAVE; ++i) r[j] += s_red[j][i];
    o.count = (u32)(total + ovf);
    o.nhub = 0;
    o.edges = r[0];
    o.in_edges = r[1];
    o.ld = r[2];
    o.ld2 = r[3];
    o.scanned = r[4];
    o.ntiles = 0;
    o.total_e = 0;
    o.decision = -1;
    o.fallback = 0;
  }
}

// ------------------------------------------------------------- edge claim
// Processes edge (u -> v) of the frontier vertex u.
template <bool ATOM>
__device__ __forceinline__ void visit_edge(const StepArgs &a, int u, int v, NewStats &st) {
  const u64 bit = 1ull << (v & 63);
  u64 *wp = a.vis + (v >> 6);
  if (ATOM) {
    bool win = false;
    u64 seen = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(seen & bit)) win = !(atomicOr(wp, bit) & bit);
    if (win) {
      a.levels[v] = a.k + 1;
      if (a.parents) a.parents[v] = u;
      atomicOr(a.fb_next + (v >> 6), bit);
      st.add_vertex(a, v);
    }
    queue_push(win, v, a);
  } else {
    if (!(*wp & bit)) {
      a.levels[v] = a.k + 1;
      if (a.parents) a.parents[v] = u;
    }
  }
}

// ------------------------------------------------ push, thread-mapped (V2)
template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_q_thread(StepArgs a) {
  __shared__ int s_seg[NSH + 2];
  clear_dead(a);
  stage_seg(s_seg, a.seg_cur);
  NewStats st;
  const int count = (int)a.c_cur->count;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
    const int u = a.q_cur[queue_slot(s_seg, a.qcap, i)];
    const int e1 = a.rp[u + 1];
    for (int j = a.rp[u]; j < e1; ++j) {
      visit_edge<ATOM>(a, u, a.ci[j], st);
      st.scanned++;
    }
  }
  st.flush(a.sh_next);
}

// Position of edge e in a staged, flattened chunk: first j with incl[j] > e.
__device__ __forceinline__ int find_owner(const int *incl, int m, int e) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (incl[mid] > e) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// ------------------------------------------- push, block-mapped (V1) + hubs
template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_q_block(StepArgs a) {
  __shared__ int s_incl[BLOCK], s_u[BLOCK], s_off[BLOCK], s_w[BLOCK / WAVE];
  __shared__ int s_seg[NSH + 2];
  clear_dead(a);
  stage_seg(s_seg, a.seg_cur);
  NewStats st;
  const int count = (int)a.c_cur->count;
  for (int c0 = blockIdx.x * BLOCK; c0 < count; c0 += gridDim.x * BLOCK) {
    const int i = c0 + threadIdx.x;
    int u = -1, beg = 0, d = 0;
    if (i < count) {
      u = a.q_cur[queue_slot(s_seg, a.qcap, i)];
      beg = a.rp[u];
      d = a.rp[u + 1] - beg;
    }
    const bool hub = d > a.hub;
    int pos = wave_append(hub, &a.c_cur->nhub);
    if (hub) {
      a.hubs[pos] = u;
      d = 0;
    }
    int total;
    int excl = block_excl_scan(d, &total, s_w);
    s_incl[threadIdx.x] = excl + d;
    s_u[threadIdx.x] = u;
    s_off[threadIdx.x] = beg - excl;
    __syncthreads();
    for (int e = threadIdx.x; e < total; e += BLOCK) {
      int j = find_owner(s_incl, BLOCK, e);
      visit_edge<ATOM>(a, s_u[j], a.ci[s_off[j] + e], st);
      st.scanned++;
    }
    __syncthreads();
  }
  st.flush(a.sh_next);
}

// Hub list of the current level, split across the whole grid: groups of 256
// hubs are flattened in LDS by every block, and block b takes edges
// b*256 + tid, stepping by the grid size.
template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_hubs(StepArgs a) {
  __shared__ int s_incl[BLOCK], s_u[BLOCK], s_off[BLOCK], s_w[BLOCK / WAVE];
  NewStats st;
  const int nhub = (int)a.c_cur->nhub;
  for (int g0 = 0; g0 < nhub; g0 += BLOCK) {
    const int h = g0 + threadIdx.x;
    int u = -1, beg = 0, d = 0;
    if (h < nhub) {
      u = a.hubs[h];
      beg = a.rp[u];
      d = a.rp[u + 1] - beg;
    }
    int total;
    int excl = block_excl_scan(d, &total, s_w);
    s_incl[threadIdx.x] = excl + d;
    s_u[threadIdx.x] = u;
    s_off[threadIdx.x] = beg - excl;
    __syncthreads();
    for (int e = blockIdx.x * BLOCK + threadIdx.x; e < total; e += gridDim.x * BLOCK) {
      int j = find_owner(s_incl, BLOCK, e);
      visit_edge<ATOM>(a, s_u[j], a.ci[s_off[j] + e], st);
      st.scanned++;
    }
    __syncthreads();
  }
  st.flush(a.sh_next);
}

// ------------------------------------------------------ push, merge path (V3)
// Pass 1: inclusive degree scan inside chunks of SCAN_CHUNK queue entries.
__global__ __launch_bounds__(BLOCK) void k_merge_scan_local(StepArgs a) {
  __shared__ int s_w[BLOCK / WAVE];
  __shared__ int s_seg[NSH + 2];
  clear_dead(a);
  stage_seg(s_seg, a.seg_cur);
  constexpr int IT = SCAN_CHUNK / BLOCK;
  const int count = (int)a.c_cur->count;
  const int nchunk = (count + SCAN_CHUNK - 1) / SCAN_CHUNK;
  for (int c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const int base = c * SCAN_CHUNK + threadIdx.x * IT;
    int d[IT];
    int run = 0;
#pragma unroll
    for (int t = 0; t < IT; ++t) {
      int i = base + t;
      int dd = 0;
      if (i < count) {
        int u = a.q_cur[queue_slot(s_seg, a.qcap, i)];
        dd = a.rp[u + 1] - a.rp[u];
      }
      run += dd;
      d[t] = run;
    }
    int total;
    int off = block_excl_scan(run, &total, s_w);
#pragma unroll
    for (int t = 0; t < IT; ++t)
      if (base + t < count) a.scan[base + t] = off + d[t];
    if (threadIdx.x == 0) a.bsum[c] = total;
  }
}

// Pass 2 (one workgroup): exclusive prefix of the chunk totals, the frontier's
// edge total and the tile count.
__global__ __launch_bounds__(BLOCK) void k_merge_scan_chunks(StepArgs a) {
  __shared__ int s_w[BLOCK / WAVE];
  const int count = (int)a.c_cur->count;
  const int nchunk = (count + SCAN_CHUNK - 1) / SCAN_CHUNK;
  int carry = 0;
  for (int c0 = 0; c0 < nchunk; c0 += BLOCK) {
    int c = c0 + threadIdx.x;
    int x = (c < nchunk) ? a.bsum[c] : 0;
    int total;
    int ex = block_excl_scan(x, &total, s_w);
    if (c < nchunk) a.bsum[c] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    a.c_cur->total_e = (u32)carry;
    a.c_cur->ntiles = (u32)((carry + MERGE_TILE - 1) / MERGE_TILE);
  }
}

__device__ __forceinline__ int merge_incl(const StepArgs &a, int i) {
  return a.scan[i] + a.bsum[i / SCAN_CHUNK];
}

// First index i in [0, count) with incl(i) > e (count when none), by a 64-ary
// search run by one whole wave.
__device__ __forceinline__ int wave_search_gt(const StepArgs &a, int count, int e) {
  int lo = 0, hi = count;  // answer in [lo, hi]
  while (hi - lo > 1) {
    const int len = hi - lo;
    const int step = (len + WAVE - 1) / WAVE;
    const int p = lo + lane() * step;  // sample points lo, lo+step, ...
    const bool gt = (p < hi) ? (merge_incl(a, p) > e) : true;
    u64 m = __ballot(gt);
    if (m == 0ull) {  // every sample (all < hi) has incl <= e
      lo = lo + (WAVE - 1) * step + 1;
      continue;
    }
    int f = __ffsll((long long)m) - 1;  // first sample with incl > e (0..63)
    if (f == 0) return lo;  // incl(lo) > e
    int nlo = lo + (f - 1) * step;  // incl(nlo) <= e
    int nhi = (lo + f * step < hi) ? lo + f * step : hi;
    lo = nlo + 1;
    hi = nhi;
    if (lo >= hi) return hi;
  }
  if (lo < hi && lo < count && merge_incl(a, lo) > e) return lo;
  return hi;
}

// Pass 3: each tile of MERGE_TILE edges stages its frontier entries in LDS
// and gives every lane an even share of the tile's edges.
template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_merge(StepArgs a) {
  __shared__ int s_incl[MERGE_STAGE], s_u[MERGE_STAGE], s_off[MERGE_STAGE];
  __shared__ int s_seg[NSH + 2];
  __shared__ int s_i0, s_m;
  stage_seg(s_seg, a.seg_cur);
  NewStats st;
  const int count = (int)a.c_cur->count;
  const int total = (int)a.c_cur->total_e;
  const int ntiles = (int)a.c_cur->ntiles;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int e0 = t * MERGE_TILE;
    const int e1 = min(total, e0 + MERGE_TILE);
    if (threadIdx.x < WAVE) {
      int i0 = wave_search_gt(a, count, e0);
      int i1 = wave_search_gt(a, count, e1 - 1);  // vertex owning the last edge
      if (lane() == 0) {
        s_i0 = i0;
        s_m = min(i1 - i0 + 1, MERGE_STAGE);
      }
    }
    __syncthreads();
    const int i0 = s_i0, m = s_m;
    for (int j = threadIdx.x; j < m; j += BLOCK) {
      int i = i0 + j;
      int u = a.q_cur[queue_slot(s_seg, a.qcap, i)];
      int inc = merge_incl(a, i);
      int beg = a.rp[u];
      int d = a.rp[u + 1] - beg;
      s_incl[j] = inc;
      s_u[j] = u;
      s_off[j] = beg - (inc - d);
    }
    __syncthreads();
    const int last_staged = s_incl[m - 1];
    for (int e = e0 + threadIdx.x; e < e1; e += BLOCK) {
      int u, pos;
      if (e < last_staged) {
        int j = find_owner(s_incl, m, e);
        u = s_u[j];
        pos = s_off[j] + e;
      } else {  // more zero-degree entries than the stage holds: search globally
        int lo = i0 + m, hi = count - 1;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (merge_incl(a, mid) > e) hi = mid; else lo = mid + 1;
        }
        u = a.q_cur[queue_slot(s_seg, a.qcap, lo)];
        int inc = merge_incl(a, lo);
        pos = a.rp[u] + e - (inc - (a.rp[u + 1] - a.rp[u]));
      }
      visit_edge<ATOM>(a, u, a.ci[pos], st);
      st.scanned++;
    }
    __syncthreads();
  }
  st.flush(a.sh_next);
}

// ------------------------------------------------ push, bitmap frontier (V10)
// One wave per bitmap word: the frontier members of 64 consecutive vertices
// are flattened with a wave scan; hubs go to the hub list.
template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_b(StepArgs a) {
  __shared__ int s_incl[BLOCK], s_u[BLOCK], s_off[BLOCK];
  clear_dead(a);
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  int *incl = s_incl + wv * WAVE;
  int *su = s_u + wv * WAVE;
  int *so = s_off + wv * WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  for (int w = gw; w < a.W; w += nw) {
    const u64 fw = a.fb_cur[w];
    if (fw == 0ull) continue;  // wave-uniform
    const int v = w * WAVE + lane();
    int beg = 0, d = 0;
    if ((fw >> lane()) & 1ull) {
      beg = a.rp[v];
      d = a.rp[v + 1] - beg;
    }
    const bool hub = d > a.hub;
    int pos = wave_append(hub, &a.c_cur->nhub);
    if (hub) {
      a.hubs[pos] = v;
      d = 0;
    }
    int in = wave_incl_scan(d);
    const int total = __shfl(in, WAVE - 1);
    incl[lane()] = in;
    su[lane()] = v;
    so[lane()] = beg - (in - d);
    __builtin_amdgcn_wave_barrier();
    for (int e = lane(); e < total; e += WAVE) {
      int j = find_owner(incl, WAVE, e);
      visit_edge<ATOM>(a, su[j], a.ci[so[j] + e], st);
      st.scanned++;
    }
    __builtin_amdgcn_wave_barrier();
  }
  st.flush(a.sh_next);
}

// ------------------------------ atomic-free: owner-computes frontier/visited
// Vertex v joined F_{k+1} iff it was unvisited (P_k) and now has depth k+1.
// The wave owning a word writes that word of P and of the next frontier
// bitmap, and appends the new vertices to the next queue.
__global__ __launch_bounds__(BLOCK) void k_noatom_update(StepArgs a) {
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  for (int w = gw; w < a.W; w += nw) {
    const u64 vw = a.vis[w];
    if (vw == ~0ull) continue;
    const int v = w * WAVE + lane();
    bool nw_ = false;
    if (!((vw >> lane()) & 1ull)) nw_ = (a.levels[v] == a.k + 1);
    const u64 m = __ballot(nw_);
    if (m) {
      if (lane() == 0) {
        a.vis[w] = vw | m;
        a.fb_next[w] = m;
      }
      if (nw_) st.add_vertex(a, v);
      queue_push(nw_, v, a);
    }
  }
  st.flush(a.sh_next);
}

// ---------------------------------------------------- pull over CSC, bitmap
// One wave owns one word (64 consecutive vertices).  Every unvisited lane
// first tests its first PULL_T in-neighbours with independent loads; a vertex
// still unresolved after that is scanned by the whole wave, 64 in-edges per
// iteration (one coalesced 256-byte read), with a ballot for the early exit.
// Either way the parent is the first frontier member in CSC order, and
// `scanned` counts the in-edges up to and including it (all of them when
// none is in the frontier), i.e. the sequential early-exit scan length.
constexpr int PULL_T = 4;

__global__ __launch_bounds__(BLOCK) void k_pull(StepArgs a) {
  clear_dead(a);
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  for (int w = gw; w < a.W; w += nw) {
    const u64 vw = a.vis[w];
    if (vw == ~0ull) continue;
    const int v = w * WAVE + lane();
    bool found = false, pending = false;
    int par = -1, b = 0, e = 0;
    if (!((vw >> lane()) & 1ull)) {
      b = a.cp[v];
      e = a.cp[v + 1];
      const int d = e - b;
      int u[PULL_T];
#pragma unroll
      for (int t = 0; t < PULL_T; ++t) u[t] = (t < d) ? a.cx[b + t] : -1;
      u64 wd[PULL_T];
#pragma unroll
      for (int t = 0; t < PULL_T; ++t) wd[t] = (u[t] >= 0) ? a.fb_cur[u[t] >> 6] : 0ull;
      int pos = -1;
#pragma unroll
      for (int t = PULL_T - 1; t >= 0; --t)
        if (u[t] >= 0 && ((wd[t] >> (u[t] & 63)) & 1ull)) pos = t;
      if (pos >= 0) {
        found = true;
        par = u[0];
#pragma unroll
        for (int t = 1; t < PULL_T; ++t)
          if (t == pos) par = u[t];
        st.scanned += (u64)(pos + 1);
      } else {
        st.scanned += (u64)min(d, PULL_T);
        pending = d > PULL_T;
        b += PULL_T;
      }
    }
    u64 pm = __ballot(pending);
    while (pm) {
      const int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      const int vb = __shfl(b, l), ve = __shfl(e, l);
      for (int base = vb; base < ve; base += WAVE) {
        const int j = base + lane();
        int uu = -1;
        bool hit = false;
        if (j < ve) {
          uu = a.cx[j];
          hit = test_bit(a.fb_cur, uu);
        }
        const u64 hm = __ballot(hit);
        if (hm) {
          const int f = __ffsll((long long)hm) - 1;
          const int p = __shfl(uu, f);
          if (lane() == l) {
            found = true;
            par = p;
            st.scanned += (u64)(base - vb + f + 1);
          }
          break;
        }
        if (base + WAVE >= ve && lane() == l) st.scanned += (u64)(ve - vb);
      }
    }
    const u64 m = __ballot(found);
    if (lane() == 0) {
      if (m) a.vis[w] = vw | m;
      a.fb_next[w] = m;
    }
    if (m) {
      if (found) {
        a.levels[v] = a.k + 1;
        if (a.parents) a.parents[v] = par;
        st.add_vertex(a, v);
      }
      queue_push(found, v, a);
    }
  }
  st.flush(a.sh_next);
}

// --------------------------------------------- state restore from depths
// F_k = {depth = k}, P_k = {0 <= depth <= k} (plus never-reachable vertices);
// scratch depths keep only <= k.  F_k's queue and counters go to the shards
// a.sh_next points at (the caller passes slot k's shards there).
__global__ __launch_bounds__(BLOCK) void k_state_from_depths(StepArgs a, const int *depths) {
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  const int tail = a.n & 63;
  for (int w = gw; w < a.W; w += nw) {
    const int v = w * WAVE + lane();
    int dv = (v < a.n) ? depths[v] : -1;
    bool in_p = dv >= 0 && dv <= a.k;
    bool in_f = dv == a.k;
    if (v < a.n) {
      a.levels[v] = in_p ? dv : -1;
      if (a.parents) a.parents[v] = (dv == 0) ? v : -1;
    }
    const bool dead = (v < a.n) && a.cp && (a.cp[v + 1] == a.cp[v]) && dv != 0;
    u64 pm = __ballot(in_p || dead), fm = __ballot(in_f);
    if (w == a.W - 1 && tail) pm |= ~0ull << tail;
    if (lane() == 0) {
      a.vis[w] = pm;
      const_cast<u64 *>(a.fb_cur)[w] = fm;
      a.fb_next[w] = 0;
      a.fb_dead[w] = 0;
    }
    if (in_f) st.add_vertex(a, v);
    queue_push(in_f, v, a);
  }
  st.scanned = 0;
  st.flush(a.sh_next);
}

__global__ void k_zero_u32(u32 *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ------------------------------------------------ graph-level degree sums
// Partials go to 64 separate lines (gsum[16 + 16 j]), summed by k_graph_ld_sum.
__global__ __launch_bounds__(BLOCK) void k_graph_ld(int n, const int *rp, u64 *gsum) {
  u64 s1 = 0, s2 = 0;
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < n; v += gridDim.x * BLOCK) {
    int l = ilog2p1(rp[v + 1] - rp[v]);
    s1 += (u64)l;
    s2 += (u64)(l * l);
  }
  s1 = wave_sum_u64(s1);
  s2 = wave_sum_u64(s2);
  if (lane() == 0) {
    const int j = blockIdx.x % 64;
    atomicAdd(gsum + 16 + 16 * j, s1);
    atomicAdd(gsum + 16 + 16 * j + 1, s2);
  }
}

__global__ void k_graph_ld_sum(u64 *gsum) {
  if (threadIdx.x == 0) {
    u64 a = 0, b = 0;
    for (int j = 0; j < 64; ++j) {
      a += gsum[16 + 16 * j];
      b += gsum[16 + 16 * j + 1];
    }
    gsum[0] = a;
    gsum[1] = b;
  }
}

// --------------------------------------------------------- CSR validation
// flag bit 0: bad offsets; bit 1: column id out of range.
__global__ __launch_bounds__(BLOCK) void k_validate(int n, int nnz, const int *ptr, const int *idx, u64 *flag) {
  u64 bad = 0;
  const int tid = blockIdx.x * BLOCK + threadIdx.x;
  const int nthr = gridDim.x * BLOCK;
  for (int v = tid; v <= n; v += nthr) {
    int p = ptr[v];
    if (v == 0 && p != 0) bad |= 1;
    if (v == n && p != nnz) bad |= 1;
    if (v < n && ptr[v + 1] < p) bad |= 1;
    if (p < 0 || p > nnz) bad |= 1;
  }
  for (int j = tid; j < nnz; j += nthr) {
    int c = idx[j];
    if (c < 0 || c >= n) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// ------------------------------------------------------------- launchers
static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
static inline int clampi(long long x, int lo, int hi) { return (int)(x < lo ? lo : (x > hi ? hi : x)); }

constexpr int GMAX = 4096;  // grid cap: grid-stride loops cover the rest

int min_first_grid(int W) { return clampi(cdiv(W, BLOCK * 4), 1, GMAX); }

hipError_t launch_reset(const StepArgs &a, int src, RingSlot *ring, hipStream_t s) {
  int grid = clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX);
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(BLOCK), 0, s, a, src, ring);
  hipLaunchKernelGGL(k_reset_f0, dim3(1), dim3(NSH + 64), 0, s, a, src, ring);
  return hipGetLastError();
}

hipError_t launch_finish(RingSlot *slot, int qcap, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(NSH), 0, s, slot, qcap);
  return hipGetLastError();
}

hipError_t launch_state_from_depths(const StepArgs &a, const int *depths, RingSlot *ring, hipStream_t s) {
  const int per = (int)(sizeof(RingSlot) / sizeof(u32));
  hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(BLOCK), 0, s, reinterpret_cast<u32 *>(ring), RING * per);
  StepArgs r = a;
  r.sh_next = ring[a.k % RING].sh;
  r.q_next = const_cast<int *>(a.q_cur);
  int grid = clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX);
  hipLaunchKernelGGL(k_state_from_depths, dim3(grid), dim3(BLOCK), 0, s, r, depths);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(NSH), 0, s, ring + (a.k % RING), a.qcap);
  return hipGetLastError();
}

hipError_t launch_graph_ld(int n, const int *rp, u64 *gsum, hipStream_t s) {
  int grid = clampi(cdiv(n, BLOCK * 8), 1, GMAX);
  hipLaunchKernelGGL(k_zero_u32, dim3(4), dim3(BLOCK), 0, s, reinterpret_cast<u32 *>(gsum + 16), 64 * 16 * 2);
  hipLaunchKernelGGL(k_graph_ld, dim3(grid), dim3(BLOCK), 0, s, n, rp, gsum);
  hipLaunchKernelGGL(k_graph_ld_sum, dim3(1), dim3(64), 0, s, gsum);
  return hipGetLastError();
}

hipError_t launch_validate(int n, int nnz, const int *ptr, const int *idx, u64 *flag, hipStream_t s) {
  int grid = clampi(cdiv((long long)n + nnz, BLOCK * 8), 1, GMAX);
  hipLaunchKernelGGL(k_validate, dim3(grid), dim3(BLOCK), 0, s, n, nnz, ptr, idx, flag);
  return hipGetLastError();
}

// count / edges: |F_k| and its out-edge total (known on the host after the
// previous level's read-back); they size the grids.
hipError_t launch_step(int variant, const StepArgs &a, int count, long long edges, hipStream_t s) {
  const int g0 = min_first_grid(a.W);
  const int gw = clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX);  // one wave per word
  const int gq = std::max(g0, clampi(cdiv(count, BLOCK), 1, GMAX));
  const int ghub = clampi(cdiv(edges, BLOCK * 2), 1, GMAX);
  switch (variant) {
    case BFS_V_PUSH_Q_THREAD:
      hipLaunchKernelGGL(k_push_q_thread<true>, dim3(gq), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_Q_BLOCK:
      hipLaunchKernelGGL(k_push_q_block<true>, dim3(gq), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<true>, dim3(ghub), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_Q_MERGE: {
      int nchunk = cdiv(count, SCAN_CHUNK);
      hipLaunchKernelGGL(k_merge_scan_local, dim3(std::max(g0, clampi(nchunk, 1, GMAX))), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_merge_scan_chunks, dim3(1), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_merge<true>, dim3(clampi(cdiv(edges, MERGE_TILE), 1, GMAX)), dim3(BLOCK), 0, s, a);
      break;
    }
    case BFS_V_PUSH_B_ATOMIC:
      hipLaunchKernelGGL(k_push_b<true>, dim3(std::max(g0, gw)), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<true>, dim3(ghub), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_B_NOATOMIC:
      hipLaunchKernelGGL(k_push_b<false>, dim3(std::max(g0, gw)), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<false>, dim3(ghub), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_noatom_update, dim3(gw), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_Q_NOATOMIC:
      hipLaunchKernelGGL(k_push_q_block<false>, dim3(gq), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<false>, dim3(ghub), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_noatom_update, dim3(gw), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PULL_B:
      hipLaunchKernelGGL(k_pull, dim3(std::max(g0, gw)), dim3(BLOCK), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bfs
