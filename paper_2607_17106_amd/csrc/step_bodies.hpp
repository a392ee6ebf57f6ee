// Device bodies of the level-step kernels, shared by the per-step kernels
// (step_kernels.hip: host- and device-driven level loops) and the persistent
// whole-search kernel (persist.hip).  Each body loops grid-stride over its
// work, so it runs unchanged under any grid; LDS comes in through `smem`.
// The algorithms are described at the top of step_kernels.hip.
#pragma once
#include "common.hpp"

namespace bfs {

// LDS bytes of each body
constexpr int SM_THREAD = (NSH + 2) * 4;
constexpr int SM_BLOCK = (3 * BLOCK + BLOCK / WAVE + NSH + 2) * 4;
constexpr int SM_HUBS = (3 * BLOCK + BLOCK / WAVE) * 4;
constexpr int SM_SCAN_LOCAL = (BLOCK / WAVE + NSH + 2) * 4;
constexpr int SM_SCAN_CHUNKS = (BLOCK / WAVE) * 4;
constexpr int SM_MERGE = (3 * MERGE_STAGE + NSH + 2 + 2) * 4;
constexpr int SM_PUSH_B = 3 * BLOCK * 4;
constexpr int SM_ADV_B = (3 * BLOCK + 2) * 4;
constexpr int SM_FINISH = 5 * (NSH / WAVE) * 8 + (NSH / WAVE) * 4;
constexpr int SM_MAX = SM_MERGE;
static_assert(SM_MERGE >= SM_BLOCK && SM_MERGE >= SM_FINISH, "SM_MAX must cover every body");

// ------------------------------------------------------------------ reset
// One wave per bitmap word.  Vertices without in-edges can never be
// discovered; their visited bits are set up front so no step searches them
// (their depth stays -1).  That needs in-degrees, i.e. CSC arrays (or a
// symmetric CSR passed as its own CSC).
__device__ __forceinline__ void body_reset(const StepArgs &a, int src, RingSlot *ring) {
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
  const int tid = blockIdx.x * BLOCK + threadIdx.x;  // BLOCK-wide workgroups
  const int nthr = gridDim.x * BLOCK;
  const int per = (int)(sizeof(RingSlot) / sizeof(u32));
  u32 *z = reinterpret_cast<u32 *>(ring);
  for (int i = tid; i < RING * per; i += nthr) z[i] = 0u;
  if (tid == 0) {
    const_cast<int *>(a.q_cur)[0] = src;
    *a.p3_level = -1;  // P_{-1} not kept yet
  }
}

// Writes F_0 = {src} into slot 0's total and segment offsets (after k_reset
// has zeroed the ring): the source sits alone in segment 0.
// Run by one workgroup.
__device__ __forceinline__ void body_reset_f0(const StepArgs &a, int src, RingSlot *slot0) {
  const int t = threadIdx.x;
  for (int i = t; i < NSH + 2; i += blockDim.x) slot0->seg[i] = (i == 0) ? 0 : 1;
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

// Log entry and loop-control counts of F_0 (k_reset_f0 wrote its totals).
__device__ __forceinline__ void body_log_f0(RingSlot *slot0, LevelLog *log, LoopCtl *ctl) {
  if (threadIdx.x == 0) {
    const LevelCtr &o = slot0->tot;
    LevelLog &L = log[0];
    L.count = o.count;
    L.variant = -1;
    L.edges = o.edges;
    L.in_edges = o.in_edges;
    L.ld = o.ld;
    L.ld2 = o.ld2;
    L.scanned = 0;
    L.fallback = 0;
    ctl->done = 0;
    ctl->levels = 1;
    ctl->reached = o.count;
    ctl->comp_edges = o.edges;
  }
}


// ------------------------------------------------------------- finish
// Reduces the NSH shards of one slot into its total and the queue segment
// offsets.  One workgroup of NSH threads.
// Must be run by exactly NSH threads of one workgroup.
__device__ __forceinline__ void body_finish(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl,
                                            char *smem) {
  u64 (*s_red)[NSH / WAVE] = reinterpret_cast<u64 (*)[NSH / WAVE]>(smem);
  int *s_w = reinterpret_cast<int *>(smem + 5 * (NSH / WAVE) * 8);
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
    if (k < LOGCAP) {
      LevelLog &L = log[k];
      L.count = o.count;
      L.variant = -1;
      L.edges = o.edges;
      L.in_edges = o.in_edges;
      L.ld = o.ld;
      L.ld2 = o.ld2;
      L.scanned = o.scanned;
      L.fallback = 0;
    }
    if (o.count == 0) {
      ctl->done = 1;
    } else if (!ctl->done) {
      ctl->levels = (u64)k + 1;
      ctl->reached += o.count;
      ctl->comp_edges += o.edges;
    }
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

// ------------------------------------- best-effort deduplication (variant 9)
// Per-wave LDS scratch of the advance that keeps duplicates (Table 3, variant
// 9): a 128-slot table of lane ids and the lanes' candidate vertices.
constexpr int DEDUP_SLOTS = 128;
constexpr int SM_DEDUP = (BLOCK / WAVE) * (DEDUP_SLOTS + WAVE) * 4;

// Edge (u -> v) in the atomic-free advance of variant 9.  A target still
// unvisited in P_k (which no lane changes during the advance) is a candidate:
// its depth and parent are written without atomics (every candidate writer
// stores depth k+1 and a valid parent), and it is appended to the temporary
// list with its source -- after a best-effort removal of duplicates among the
// wave's current candidates, without sorting: each candidate lane writes its
// id into the slot of its vertex's hash, and a lane whose slot names another
// lane holding the same vertex drops out.  Duplicates that survive (two
// waves, a hash collision) are removed by the filter, whose claims are exact.
// A candidate that finds the list full is claimed here as the atomic push
// claims it.  Called by the active lanes of a wave together.
__device__ __forceinline__ void visit_edge_dedup(const StepArgs &a, int u, int v, NewStats &st, int *tab, int *vals) {
  const u64 bit = 1ull << (v & 63);
  const bool cand = !(a.vis[v >> 6] & bit);
  if (cand) {
    a.levels[v] = a.k + 1;
    if (a.parents) a.parents[v] = u;
  }
  const int l = lane();
  const int h = (int)(((u32)v * 2654435761u) >> 25);  // 0 .. DEDUP_SLOTS-1
  vals[l] = v;
  if (cand) tab[h] = l;
  __builtin_amdgcn_wave_barrier();
  bool keep = cand;
  if (cand) {
    const int o = tab[h];
    if (o != l && vals[o] == v) keep = false;
  }
  __builtin_amdgcn_wave_barrier();
  const int pos = wave_append(keep, &a.c_cur->total_e);
  const bool fits = keep && pos < a.tmpcap;
  if (fits) {
    a.tmp_v[pos] = v;
    a.tmp_u[pos] = u;
  }
  if (keep && !fits) {  // the list is full: claim now
    const bool win = !(atomicOr(a.vis + (v >> 6), bit) & bit);
    if (win) {
      atomicOr(a.fb_next + (v >> 6), bit);
      st.add_vertex(a, v);
    }
    queue_push(win, v, a);
  }
}

// ------------------------------------------------ push, thread-mapped (V2)
template <bool ATOM>
__device__ __forceinline__ void body_push_q_thread(const StepArgs &a, char *smem) {
  int *s_seg = reinterpret_cast<int *>(smem);
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
template <bool ATOM, bool DEDUP = false>
__device__ __forceinline__ void body_push_q_block(const StepArgs &a, char *smem, int *dedup = nullptr) {
  int *s_incl = reinterpret_cast<int *>(smem), *s_u = s_incl + BLOCK, *s_off = s_u + BLOCK;
  int *s_w = s_off + BLOCK, *s_seg = s_w + BLOCK / WAVE;
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
      if (DEDUP)
        visit_edge_dedup(a, s_u[j], a.ci[s_off[j] + e], st, dedup + (threadIdx.x / WAVE) * (DEDUP_SLOTS + WAVE),
                         dedup + (threadIdx.x / WAVE) * (DEDUP_SLOTS + WAVE) + DEDUP_SLOTS);
      else
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
template <bool ATOM, bool DEDUP = false>
__device__ __forceinline__ void body_push_hubs(const StepArgs &a, char *smem, int *dedup = nullptr) {
  int *s_incl = reinterpret_cast<int *>(smem), *s_u = s_incl + BLOCK, *s_off = s_u + BLOCK;
  int *s_w = s_off + BLOCK;
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
      if (DEDUP)
        visit_edge_dedup(a, s_u[j], a.ci[s_off[j] + e], st, dedup + (threadIdx.x / WAVE) * (DEDUP_SLOTS + WAVE),
                         dedup + (threadIdx.x / WAVE) * (DEDUP_SLOTS + WAVE) + DEDUP_SLOTS);
      else
        visit_edge<ATOM>(a, s_u[j], a.ci[s_off[j] + e], st);
      st.scanned++;
    }
    __syncthreads();
  }
  st.flush(a.sh_next);
}

// ------------------------------------------------------ push, merge path (V3)
// Pass 1: inclusive degree scan inside chunks of SCAN_CHUNK queue entries.
__device__ __forceinline__ void body_merge_scan_local(const StepArgs &a, char *smem) {
  int *s_w = reinterpret_cast<int *>(smem), *s_seg = s_w + BLOCK / WAVE;
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

// Pass 1 over bitmap words instead (advance then filter with a bitmap
// frontier, Table 3, variant 14): entry w weighs the out-degrees of the
// frontier members in word w of F_k.
__device__ __forceinline__ void body_wscan_local(const StepArgs &a, char *smem) {
  int *s_w = reinterpret_cast<int *>(smem);
  constexpr int IT = SCAN_CHUNK / BLOCK;
  const int nchunk = (a.W + SCAN_CHUNK - 1) / SCAN_CHUNK;
  for (int c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const int base = c * SCAN_CHUNK + threadIdx.x * IT;
    int d[IT];
    int run = 0;
#pragma unroll
    for (int t = 0; t < IT; ++t) {
      const int w = base + t;
      int dd = 0;
      if (w < a.W) {
        for (u64 fw = a.fb_cur[w]; fw; fw &= fw - 1) {
          const int v = w * WAVE + __ffsll((long long)fw) - 1;
          dd += a.rp[v + 1] - a.rp[v];
        }
      }
      run += dd;
      d[t] = run;
    }
    int total;
    int off = block_excl_scan(run, &total, s_w);
#pragma unroll
    for (int t = 0; t < IT; ++t)
      if (base + t < a.W) a.scan[base + t] = off + d[t];
    if (threadIdx.x == 0) a.bsum[c] = total;
  }
}

// Pass 2 (one workgroup): exclusive prefix of the chunk totals, the frontier's
// edge total and the tile count, over `count` entries (queue entries, or
// bitmap words when count < 0).
// Runs in workgroup 0 only (other workgroups return at once).
__device__ __forceinline__ void body_merge_scan_chunks(const StepArgs &a, char *smem, bool words = false) {
  if (blockIdx.x != 0) return;
  int *s_w = reinterpret_cast<int *>(smem);
  const int count = words ? a.W : (int)a.c_cur->count;
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
// TMP (advance before the depth update, Table 3, variant 13): only the edges
// [chunk * tmpcap, (chunk + 1) * tmpcap) of the flattened list, each written
// with its source to the temporary list at its offset in the chunk; no
// visited test and no atomics.
template <bool ATOM, bool TMP = false>
__device__ __forceinline__ void body_push_merge(const StepArgs &a, char *smem, int chunk = 0) {
  int *s_incl = reinterpret_cast<int *>(smem), *s_u = s_incl + MERGE_STAGE, *s_off = s_u + MERGE_STAGE;
  int *s_seg = s_off + MERGE_STAGE;
  int &s_i0 = s_seg[NSH + 2], &s_m = s_seg[NSH + 3];
  stage_seg(s_seg, a.seg_cur);
  NewStats st;
  const int count = (int)a.c_cur->count;
  const int e_lo = TMP ? chunk * a.tmpcap : 0;
  const int total = TMP ? (int)min((long long)a.c_cur->total_e, (long long)e_lo + a.tmpcap) : (int)a.c_cur->total_e;
  const int t_lo = e_lo / MERGE_TILE;
  const int ntiles = TMP ? (total > e_lo ? (total + MERGE_TILE - 1) / MERGE_TILE : t_lo) : (int)a.c_cur->ntiles;
  for (int t = t_lo + blockIdx.x; t < ntiles; t += gridDim.x) {
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
      if (TMP) {
        a.tmp_v[e - e_lo] = a.ci[pos];
        a.tmp_u[e - e_lo] = u;
      } else {
        visit_edge<ATOM>(a, u, a.ci[pos], st);
      }
      st.scanned++;
    }
    __syncthreads();
  }
  st.flush(a.sh_next);
}

// Advance of variant 14: the edges [chunk * tmpcap, (chunk + 1) * tmpcap) of
// the flattened list of the bitmap frontier's out-edges (word by word, bits
// in order) go to the temporary list at their offset in the chunk.  A tile of
// MERGE_TILE edges finds its first and last word by the 64-ary wave search;
// its waves take those words in turn and write only the tile's positions of
// each, so a word holding a hub is split across as many tiles as it spans.
__device__ __forceinline__ void body_adv_tmp_b(const StepArgs &a, char *smem, int chunk) {
  int *s_incl = reinterpret_cast<int *>(smem), *s_u = s_incl + BLOCK, *s_off = s_u + BLOCK;
  int *s_rng = s_off + BLOCK;
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  int *incl = s_incl + wv * WAVE;
  int *su = s_u + wv * WAVE;
  int *so = s_off + wv * WAVE;
  const int e_lo = chunk * a.tmpcap;
  const int total = (int)min((long long)a.c_cur->total_e, (long long)e_lo + a.tmpcap);
  const int t_lo = e_lo / MERGE_TILE;
  const int ntiles = total > e_lo ? (total + MERGE_TILE - 1) / MERGE_TILE : t_lo;
  for (int t = t_lo + blockIdx.x; t < ntiles; t += gridDim.x) {
    const int e0 = t * MERGE_TILE;
    const int e1 = min(total, e0 + MERGE_TILE);
    if (threadIdx.x < WAVE) {
      const int w0 = wave_search_gt(a, a.W, e0);
      const int w1 = wave_search_gt(a, a.W, e1 - 1);
      if (lane() == 0) {
        s_rng[0] = w0;
        s_rng[1] = w1;
      }
    }
    __syncthreads();
    const int w0 = s_rng[0], w1 = s_rng[1];
    for (int w = w0 + wv; w <= w1; w += BLOCK / WAVE) {  // uniform per wave
      const u64 fw = a.fb_cur[w];
      const int wend = merge_incl(a, w);  // flattened edges before the end of word w
      const int v = w * WAVE + lane();
      int beg = 0, d = 0;
      if ((fw >> lane()) & 1ull) {
        beg = a.rp[v];
        d = a.rp[v + 1] - beg;
      }
      const int in = wave_incl_scan(d);
      const int wt = lane_bcast(in, WAVE - 1);
      const int wbase = wend - wt;
      incl[lane()] = in;
      su[lane()] = v;
      so[lane()] = beg - (in - d);
      __builtin_amdgcn_wave_barrier();
      const int lo = max(e0, wbase) - wbase, hi = min(e1, wend) - wbase;
      for (int e = lo + lane(); e < hi; e += WAVE) {
        const int j = find_owner(incl, WAVE, e);
        a.tmp_v[wbase + e - e_lo] = a.ci[so[j] + e];
        a.tmp_u[wbase + e - e_lo] = su[j];
        st.scanned++;
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
  st.flush(a.sh_next);
}

// Filter of variant 13: claims the entries of one chunk of the temporary list
// as the atomic push claims an edge (visited test, depth, parent, F_{k+1}).
__device__ __forceinline__ void body_filter_tmp(const StepArgs &a, int chunk) {
  NewStats st;
  const long long e_lo = (long long)chunk * a.tmpcap;
  const int len = (int)max(0ll, min((long long)a.c_cur->total_e - e_lo, (long long)a.tmpcap));
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < len; i += gridDim.x * BLOCK)
    visit_edge<true>(a, a.tmp_u[i], a.tmp_v[i], st);
  st.flush(a.sh_next);
}

// ------------------------------------------------ push, bitmap frontier (V10)
// One wave per bitmap word: the frontier members of 64 consecutive vertices
// are flattened with a wave scan; hubs go to the hub list.
template <bool ATOM>
__device__ __forceinline__ void body_push_b(const StepArgs &a, char *smem) {
  int *s_incl = reinterpret_cast<int *>(smem), *s_u = s_incl + BLOCK, *s_off = s_u + BLOCK;
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
    const int total = lane_bcast(in, WAVE - 1);
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
__device__ __forceinline__ void body_noatom_update(const StepArgs &a) {
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

// ------------------------------ three visited arrays (Table 3, variant 26)
// The frontier is not kept as an array of its own: F_k = P_k AND NOT P_{k-1}
// (the three arrays are P_{k-1}, P_k and the P_{k+1} the update builds in
// place).  The expansion is atomic-free as in body_push_b<false>; when the
// previous level was run by another variant P_{k-1} is not at hand and the
// frontier bitmap every step emits stands in for one level.
__device__ __forceinline__ void body_push_p3(const StepArgs &a, char *smem) {
  int *s_incl = reinterpret_cast<int *>(smem), *s_u = s_incl + BLOCK, *s_off = s_u + BLOCK;
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  int *incl = s_incl + wv * WAVE;
  int *su = s_u + wv * WAVE;
  int *so = s_off + wv * WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  const bool derive = *a.p3_level == a.k;
  for (int w = gw; w < a.W; w += nw) {
    const u64 fw = derive ? (a.vis[w] & ~a.vis_prev[w]) : a.fb_cur[w];
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
    const int total = lane_bcast(in, WAVE - 1);
    incl[lane()] = in;
    su[lane()] = v;
    so[lane()] = beg - (in - d);
    __builtin_amdgcn_wave_barrier();
    for (int e = lane(); e < total; e += WAVE) {
      int j = find_owner(incl, WAVE, e);
      visit_edge<false>(a, su[j], a.ci[so[j] + e], st);
      st.scanned++;
    }
    __builtin_amdgcn_wave_barrier();
  }
  st.flush(a.sh_next);
}

// Owner computes, as body_noatom_update, and keeps P_k as the next level's
// P_{k-1}: every word of vis_prev is rewritten, then the level tag.
__device__ __forceinline__ void body_p3_update(const StepArgs &a) {
  NewStats st;
  const int wv = threadIdx.x / WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wv;
  const int nw = gridDim.x * (BLOCK / WAVE);
  for (int w = gw; w < a.W; w += nw) {
    const u64 vw = a.vis[w];
    const int v = w * WAVE + lane();
    bool nw_ = false;
    if (vw != ~0ull && !((vw >> lane()) & 1ull)) nw_ = (a.levels[v] == a.k + 1);
    const u64 m = __ballot(nw_);
    if (lane() == 0) {
      a.vis_prev[w] = vw;
      if (m) {
        a.vis[w] = vw | m;
        a.fb_next[w] = m;
      }
    }
    if (m) {
      if (nw_) st.add_vertex(a, v);
      queue_push(nw_, v, a);
    }
  }
  st.flush(a.sh_next);
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.p3_level = a.k + 1;
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

// FROM_VIS (Table 3, variant 25: visited as frontier): the
// in-neighbour test reads the visited set P_k instead of the frontier.  Every
// member of P_k that is an in-neighbour of a vertex still unvisited after
// level k is at depth k (one at depth j < k would have reached it at j + 1),
// so the first visited in-neighbour is the first frontier in-neighbour: same
// depths, same parents, same scan lengths.  The visited bitmap also holds
// vertices marked only because they can never be reached (in-degree 0, or
// unreachable in a restored state); their depth is -1, so a bitmap hit counts
// only when the depth is set.  P_k must stay fixed during the step, so the
// new bits go to the next bitmap only and body_merge_vis folds them into the
// visited bitmap afterwards.
template <bool FROM_VIS>
__device__ __forceinline__ void body_pull(const StepArgs &a) {
  const u64 *front = FROM_VIS ? a.vis : a.fb_cur;
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
      for (int t = 0; t < PULL_T; ++t) wd[t] = (u[t] >= 0) ? front[u[t] >> 6] : 0ull;
      bool hb[PULL_T];
#pragma unroll
      for (int t = 0; t < PULL_T; ++t) hb[t] = u[t] >= 0 && ((wd[t] >> (u[t] & 63)) & 1ull);
      if (FROM_VIS) {
#pragma unroll
        for (int t = 0; t < PULL_T; ++t) hb[t] = hb[t] && a.levels[u[t]] >= 0;
      }
      int pos = -1;
#pragma unroll
      for (int t = PULL_T - 1; t >= 0; --t)
        if (hb[t]) pos = t;
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
      const int vb = lane_bcast(b, l), ve = lane_bcast(e, l);
      for (int base = vb; base < ve; base += WAVE) {
        const int j = base + lane();
        int uu = -1;
        bool hit = false;
        if (j < ve) {
          uu = a.cx[j];
          hit = test_bit(front, uu);
          if (FROM_VIS && hit) hit = a.levels[uu] >= 0;
        }
        const u64 hm = __ballot(hit);
        if (hm) {
          const int f = __ffsll((long long)hm) - 1;
          const int p = lane_bcast(uu, f);
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
      if (m && !FROM_VIS) a.vis[w] = vw | m;
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

// After a visited-as-frontier pull: P_{k+1} = P_k OR F_{k+1}.
__device__ __forceinline__ void body_merge_vis(const StepArgs &a) {
  for (int w = blockIdx.x * BLOCK + threadIdx.x; w < a.W; w += gridDim.x * BLOCK) {  // BLOCK-wide workgroups
    const u64 m = a.fb_next[w];
    if (m) a.vis[w] |= m;
  }
}

}  // namespace bfs
