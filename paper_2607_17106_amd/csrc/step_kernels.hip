// Level-step kernels of single-source BFS for gfx950 (wave64).
//
// One level expands F_k into F_{k+1} (Cascade 1, Eq. advance) and merges it
// into the visited set P (Eq. update).  Layout: visited P and frontier
// bitmaps are u64 words (bit v&63 of word v>>6); frontier queues are int32
// vertex lists; depths/parents are int32 per vertex.
//
// Push (top-down) kernels walk out-edges of F_k (loop order s -> d, Sec.
// "The Einsum-Enabled Design Space", B.1) and claim each unvisited d:
//   ATOM = true : one atomicOr on d's visited word decides the single winner,
//                 which writes depth/parent and appends d (Table 3, variant 1-3, 10).
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
#include "common.hpp"

namespace bfs {

// ------------------------------------------------------------------ reset
__global__ void k_reset(StepArgs a, int src) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthr = gridDim.x * blockDim.x;
  for (int v = tid; v < a.n; v += nthr) {
    a.levels[v] = (v == src) ? 0 : -1;
    if (a.parents) a.parents[v] = (v == src) ? src : -1;
  }
  const int tail = a.n & 63;
  for (int w = tid; w < a.W; w += nthr) {
    u64 vw = 0;
    if (w == (src >> 6)) vw |= 1ull << (src & 63);
    u64 fw = vw;
    if (w == a.W - 1 && tail) vw |= ~0ull << tail;  // bits >= n count as visited
    a.vis[w] = vw;
    a.fb_next[w] = 0;  // fb[0] = current (holds the source), fb[1] next, fb[2] dead
    a.fb_dead[w] = 0;
    const_cast<u64 *>(a.fb_cur)[w] = fw;
  }
  if (tid == 0) const_cast<int *>(a.q_cur)[0] = src;
  if (tid < RING * (int)(sizeof(LevelCtr) / sizeof(u32))) {
    reinterpret_cast<u32 *>(a.c_cur)[tid] = 0u;  // c_cur is slot 0 of the ring
  }
  __syncthreads();
  if (tid == 0) {
    int d = a.rp[src + 1] - a.rp[src];
    int di = a.cp ? a.cp[src + 1] - a.cp[src] : d;
    int l = ilog2p1(d);
    a.c_cur->count = 1;
    a.c_cur->edges = (u64)d;
    a.c_cur->in_edges = (u64)di;
    a.c_cur->ld = (u64)l;
    a.c_cur->ld2 = (u64)(l * l);
  }
}

// ------------------------------------------------------------- edge claim
// Processes edge (u -> v) of the frontier vertex u.
template <bool ATOM>
__device__ __forceinline__ void visit_edge(const StepArgs &a, int u, int v, NewStats &st) {
  const u64 bit = 1ull << (v & 63);
  u64 *wp = a.vis + (v >> 6);
  bool win = false;
  if (ATOM) {
    u64 seen = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(seen & bit)) win = !(atomicOr(wp, bit) & bit);
    if (win) {
      a.levels[v] = a.k + 1;
      if (a.parents) a.parents[v] = u;
      atomicOr(a.fb_next + (v >> 6), bit);
      st.add_vertex(a, v);
    }
    int pos = wave_append(win, &a.c_next->count);
    if (win) a.q_next[pos] = v;
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
  clear_dead(a);
  NewStats st;
  const int count = (int)a.c_cur->count;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
    const int u = a.q_cur[i];
    const int e1 = a.rp[u + 1];
    for (int j = a.rp[u]; j < e1; ++j) {
      visit_edge<ATOM>(a, u, a.ci[j], st);
      st.scanned++;
    }
  }
  st.flush(a.c_next);
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
  clear_dead(a);
  NewStats st;
  const int count = (int)a.c_cur->count;
  for (int c0 = blockIdx.x * BLOCK; c0 < count; c0 += gridDim.x * BLOCK) {
    const int i = c0 + threadIdx.x;
    int u = -1, beg = 0, d = 0;
    if (i < count) {
      u = a.q_cur[i];
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
  st.flush(a.c_next);
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
  st.flush(a.c_next);
}

// ------------------------------------------------------ push, merge path (V3)
// Pass 1: inclusive degree scan inside chunks of SCAN_CHUNK queue entries.
__global__ __launch_bounds__(BLOCK) void k_merge_scan_local(StepArgs a) {
  __shared__ int s_w[BLOCK / WAVE];
  clear_dead(a);
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
        int u = a.q_cur[i];
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
  __shared__ int s_i0, s_m;
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
      int u = a.q_cur[i];
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
        int i = i0 + m;
        int lo = i, hi = count - 1;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (merge_incl(a, mid) > e) hi = mid; else lo = mid + 1;
        }
        u = a.q_cur[lo];
        int inc = merge_incl(a, lo);
        pos = a.rp[u] + e - (inc - (a.rp[u + 1] - a.rp[u]));
      }
      visit_edge<ATOM>(a, u, a.ci[pos], st);
      st.scanned++;
    }
    __syncthreads();
  }
  st.flush(a.c_next);
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
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (int e = lane(); e < total; e += WAVE) {
      int j = find_owner(incl, WAVE, e);
      visit_edge<ATOM>(a, su[j], a.ci[so[j] + e], st);
      st.scanned++;
    }
    __builtin_amdgcn_wave_barrier();
  }
  st.flush(a.c_next);
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
      int pos = wave_append(nw_, &a.c_next->count);
      if (nw_) a.q_next[pos] = v;
    }
  }
  st.flush(a.c_next);
}

// ---------------------------------------------------- pull over CSC, bitmap
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
    bool found = false;
    int par = -1;
    if (!((vw >> lane()) & 1ull)) {
      const int j1 = a.cp[v + 1];
      for (int j = a.cp[v]; j < j1; ++j) {
        const int u = a.cx[j];
        st.scanned++;
        if (test_bit(a.fb_cur, u)) {
          found = true;
          par = u;
          break;
        }
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
      int pos = wave_append(found, &a.c_next->count);
      if (found) a.q_next[pos] = v;
    }
  }
  st.flush(a.c_next);
}

// --------------------------------------------- state restore from depths
// F_k = {depth = k}, P_k = {0 <= depth <= k}; scratch depths keep only <= k.
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
    u64 pm = __ballot(in_p), fm = __ballot(in_f);
    if (w == a.W - 1 && tail) pm |= ~0ull << tail;
    if (lane() == 0) {
      a.vis[w] = pm;
      const_cast<u64 *>(a.fb_cur)[w] = fm;
      a.fb_next[w] = 0;
      a.fb_dead[w] = 0;
    }
    if (in_f) st.add_vertex(a, v);
    int pos = wave_append(in_f, &a.c_cur->count);
    if (in_f) const_cast<int *>(a.q_cur)[pos] = v;
  }
  st.scanned = 0;
  st.flush(a.c_cur);
}

__global__ void k_zero_ring(LevelCtr *c) {
  if (threadIdx.x < RING * (int)(sizeof(LevelCtr) / sizeof(u32))) reinterpret_cast<u32 *>(c)[threadIdx.x] = 0u;
}

// ------------------------------------------------ graph-level degree sums
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
    atomicAdd(gsum + 0, s1);
    atomicAdd(gsum + 1, s2);
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

int min_first_grid(int W) { return cdiv(W, BLOCK * 4); }

hipError_t launch_reset(const StepArgs &a, int src, hipStream_t s) {
  int grid = clampi(cdiv(a.n, BLOCK * 4), 1, 8192);
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(BLOCK), 0, s, a, src);
  return hipGetLastError();
}

hipError_t launch_state_from_depths(const StepArgs &a, const int *depths, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ring, dim3(1), dim3(BLOCK), 0, s, a.c_cur - (a.k % RING));
  int grid = clampi(cdiv(a.W, BLOCK / WAVE), 1, 16384);
  hipLaunchKernelGGL(k_state_from_depths, dim3(grid), dim3(BLOCK), 0, s, a, depths);
  return hipGetLastError();
}

hipError_t launch_graph_ld(int n, const int *rp, u64 *gsum, hipStream_t s) {
  int grid = clampi(cdiv(n, BLOCK * 8), 1, 4096);
  hipLaunchKernelGGL(k_graph_ld, dim3(grid), dim3(BLOCK), 0, s, n, rp, gsum);
  return hipGetLastError();
}

hipError_t launch_validate(int n, int nnz, const int *ptr, const int *idx, u64 *flag, hipStream_t s) {
  int grid = clampi(cdiv((long long)n + nnz, BLOCK * 8), 1, 4096);
  hipLaunchKernelGGL(k_validate, dim3(grid), dim3(BLOCK), 0, s, n, nnz, ptr, idx, flag);
  return hipGetLastError();
}

// count / edges: |F_k| and its out-edge total (known on the host after the
// previous level's read-back); they size the grids.
hipError_t launch_step(int variant, const StepArgs &a, int count, long long edges, hipStream_t s) {
  const int g0 = min_first_grid(a.W);
  const int gw = clampi(cdiv(a.W, BLOCK / WAVE), 1, 8192);  // one wave per word
  const int ghub = clampi(cdiv(edges, BLOCK * 16), 1, 2048);
  switch (variant) {
    case BFS_V_PUSH_Q_THREAD:
      hipLaunchKernelGGL(k_push_q_thread<true>, dim3(std::max(g0, clampi(cdiv(count, BLOCK), 1, 65536))),
                         dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_Q_BLOCK:
      hipLaunchKernelGGL(k_push_q_block<true>, dim3(std::max(g0, clampi(cdiv(count, BLOCK), 1, 65536))),
                         dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<true>, dim3(ghub), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_Q_MERGE: {
      int nchunk = cdiv(count, SCAN_CHUNK);
      hipLaunchKernelGGL(k_merge_scan_local, dim3(std::max(g0, clampi(nchunk, 1, 65536))), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_merge_scan_chunks, dim3(1), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_merge<true>, dim3(clampi(cdiv(edges, MERGE_TILE), 1, 65536)), dim3(BLOCK), 0, s, a);
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
      hipLaunchKernelGGL(k_push_q_block<false>, dim3(std::max(g0, clampi(cdiv(count, BLOCK), 1, 65536))),
                         dim3(BLOCK), 0, s, a);
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
