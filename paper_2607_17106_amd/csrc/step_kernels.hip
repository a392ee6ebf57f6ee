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
#include "step_bodies.hpp"

namespace bfs {

// ------------------------------------------------------------------ reset
__global__ __launch_bounds__(BLOCK) void k_reset(StepArgs a, int src, RingSlot *ring) { body_reset(a, src, ring); }
__global__ void k_reset_f0(StepArgs a, int src, RingSlot *slot0) { body_reset_f0(a, src, slot0); }
__global__ void k_log_f0(RingSlot *slot0, LevelLog *log, LoopCtl *ctl) { body_log_f0(slot0, log, ctl); }

hipError_t launch_log_f0(RingSlot *slot0, LevelLog *log, LoopCtl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_log_f0, dim3(1), dim3(64), 0, s, slot0, log, ctl);
  return hipGetLastError();
}

// ------------------------------------------------------ per-step kernels
// Thin wrappers over the bodies in step_bodies.hpp: clear the dead buffers,
// check the device-loop gate, run the body.
__global__ __launch_bounds__(NSH) void k_finish(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl) {
  __shared__ __align__(16) char smem[SM_FINISH];
  body_finish(slot, qcap, k, log, ctl, smem);
}

template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_q_thread(StepArgs a) {
  __shared__ __align__(16) char smem[SM_THREAD];
  clear_dead(a);
  if (gated_off(a)) return;
  body_push_q_thread<ATOM>(a, smem);
}

template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_q_block(StepArgs a) {
  __shared__ __align__(16) char smem[SM_BLOCK];
  clear_dead(a);
  if (gated_off(a)) return;
  body_push_q_block<ATOM>(a, smem);
}

template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_hubs(StepArgs a) {
  __shared__ __align__(16) char smem[SM_HUBS];
  if (gated_off(a)) return;
  body_push_hubs<ATOM>(a, smem);
}

// advance of variant 9 (best-effort deduplication), block-mapped with hubs
// deferred, then the hubs grid-wide; the filter (k_filter_tmp) claims
__global__ __launch_bounds__(BLOCK) void k_push_q_dedup(StepArgs a) {
  __shared__ __align__(16) char smem[SM_BLOCK];
  __shared__ int s_dedup[SM_DEDUP / 4];
  clear_dead(a);
  if (gated_off(a)) return;
  body_push_q_block<false, true>(a, smem, s_dedup);
}

__global__ __launch_bounds__(BLOCK) void k_push_hubs_dedup(StepArgs a) {
  __shared__ __align__(16) char smem[SM_HUBS];
  __shared__ int s_dedup[SM_DEDUP / 4];
  if (gated_off(a)) return;
  body_push_hubs<false, true>(a, smem, s_dedup);
}

__global__ __launch_bounds__(BLOCK) void k_merge_scan_local(StepArgs a) {
  __shared__ __align__(16) char smem[SM_SCAN_LOCAL];
  clear_dead(a);
  if (gated_off(a)) return;
  body_merge_scan_local(a, smem);
}

__global__ __launch_bounds__(BLOCK) void k_wscan_local(StepArgs a) {
  __shared__ __align__(16) char smem[SM_SCAN_LOCAL];
  clear_dead(a);
  if (gated_off(a)) return;
  body_wscan_local(a, smem);
}

__global__ __launch_bounds__(BLOCK) void k_wscan_chunks(StepArgs a) {
  __shared__ __align__(16) char smem[SM_SCAN_CHUNKS];
  if (gated_off(a)) return;
  body_merge_scan_chunks(a, smem, true);
}

__global__ __launch_bounds__(BLOCK) void k_adv_tmp_b(StepArgs a, int chunk) {
  __shared__ __align__(16) char smem[SM_ADV_B];
  if (gated_off(a)) return;
  body_adv_tmp_b(a, smem, chunk);
}

__global__ __launch_bounds__(BLOCK) void k_merge_scan_chunks(StepArgs a) {
  __shared__ __align__(16) char smem[SM_SCAN_CHUNKS];
  if (gated_off(a)) return;
  body_merge_scan_chunks(a, smem);
}

template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_merge(StepArgs a) {
  __shared__ __align__(16) char smem[SM_MERGE];
  if (gated_off(a)) return;
  body_push_merge<ATOM>(a, smem);
}

template <bool ATOM>
__global__ __launch_bounds__(BLOCK) void k_push_b(StepArgs a) {
  __shared__ __align__(16) char smem[SM_PUSH_B];
  clear_dead(a);
  if (gated_off(a)) return;
  body_push_b<ATOM>(a, smem);
}

__global__ __launch_bounds__(BLOCK) void k_noatom_update(StepArgs a) {
  if (gated_off(a)) return;
  body_noatom_update(a);
}

// advance then filter (Table 3, variant 13), one chunk of the temporary list
__global__ __launch_bounds__(BLOCK) void k_adv_tmp(StepArgs a, int chunk) {
  __shared__ __align__(16) char smem[SM_MERGE];
  if (gated_off(a)) return;
  body_push_merge<true, true>(a, smem, chunk);
}

__global__ __launch_bounds__(BLOCK) void k_filter_tmp(StepArgs a, int chunk) {
  if (gated_off(a)) return;
  body_filter_tmp(a, chunk);
}

__global__ __launch_bounds__(BLOCK) void k_push_p3(StepArgs a) {
  __shared__ __align__(16) char smem[SM_PUSH_B];
  clear_dead(a);
  if (gated_off(a)) return;
  body_push_p3(a, smem);
}

__global__ __launch_bounds__(BLOCK) void k_p3_update(StepArgs a) {
  if (gated_off(a)) return;
  body_p3_update(a);
}

template <bool FROM_VIS>
__global__ __launch_bounds__(BLOCK) void k_pull(StepArgs a) {
  clear_dead(a);
  if (gated_off(a)) return;
  body_pull<FROM_VIS>(a);
}

__global__ __launch_bounds__(BLOCK) void k_merge_vis(StepArgs a) {
  if (gated_off(a)) return;
  body_merge_vis(a);
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
    u64 pm = __ballot(in_p || dead), fm = __ballot(in_f), qm = __ballot((in_p && !in_f) || dead);
    if (w == a.W - 1 && tail) {
      pm |= ~0ull << tail;
      qm |= ~0ull << tail;
    }
    if (lane() == 0) {
      a.vis[w] = pm;
      a.vis_prev[w] = qm;  // P_{k-1}, for the three-array variant
      const_cast<u64 *>(a.fb_cur)[w] = fm;
      a.fb_next[w] = 0;
      a.fb_dead[w] = 0;
    }
    if (in_f) st.add_vertex(a, v);
    queue_push(in_f, v, a);
  }
  st.scanned = 0;
  st.flush(a.sh_next);
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.p3_level = a.k;
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

hipError_t launch_reset(const StepArgs &a, int src, RingSlot *ring, hipStream_t s, bool f0) {
  int grid = clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX);
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(BLOCK), 0, s, a, src, ring);
  if (f0) hipLaunchKernelGGL(k_reset_f0, dim3(1), dim3(NSH + 64), 0, s, a, src, ring);
  return hipGetLastError();
}

hipError_t launch_finish(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(NSH), 0, s, slot, qcap, k, log, ctl);
  return hipGetLastError();
}

// The state restore's finish needs a LoopCtl it may scribble on: the pad of
// the last ring slot serves.
static LoopCtl *scratch_ctl(RingSlot *ring) {
  return reinterpret_cast<LoopCtl *>(ring[RING - 1].pad);
}

hipError_t launch_state_from_depths(const StepArgs &a, const int *depths, RingSlot *ring, hipStream_t s) {
  const int per = (int)(sizeof(RingSlot) / sizeof(u32));
  hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(BLOCK), 0, s, reinterpret_cast<u32 *>(ring), RING * per);
  StepArgs r = a;
  r.sh_next = ring[a.k % RING].sh;
  r.q_next = const_cast<int *>(a.q_cur);
  int grid = clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX);
  hipLaunchKernelGGL(k_state_from_depths, dim3(grid), dim3(BLOCK), 0, s, r, depths);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(NSH), 0, s, ring + (a.k % RING), a.qcap, LOGCAP, (LevelLog *)nullptr,
                     scratch_ctl(ring));
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
constexpr int GDEV = 1024;  // device loop: grid when sizes are unknown on the host

hipError_t launch_step(int variant, const StepArgs &a, int count, long long edges, hipStream_t s) {
  const bool dev = count < 0;
  const int g0 = min_first_grid(a.W);
  const int gw = dev ? std::min(GDEV, clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX)) : clampi(cdiv(a.W, BLOCK / WAVE), 1, GMAX);
  const int gq = dev ? std::max(g0, GDEV) : std::max(g0, clampi(cdiv(count, BLOCK), 1, GMAX));
  const int ghub = dev ? GDEV : clampi(cdiv(edges, BLOCK * 2), 1, GMAX);
  if (dev) {
    count = GDEV * SCAN_CHUNK;
    edges = (long long)GDEV * MERGE_TILE;
  }
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
    case BFS_V_PUSH_Q_DEDUP: {
      // candidates (at most the frontier's out-edges, and the list's size)
      const long long span = std::min(dev ? (long long)a.nnz : edges, (long long)a.tmpcap);
      hipLaunchKernelGGL(k_push_q_dedup, dim3(gq), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs_dedup, dim3(ghub), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_filter_tmp, dim3(clampi(cdiv(std::max(span, 1ll), BLOCK), 1, GMAX)), dim3(BLOCK), 0, s, a, 0);
      break;
    }
    case BFS_V_PUSH_Q_NOATOMIC:
      hipLaunchKernelGGL(k_push_q_block<false>, dim3(gq), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<false>, dim3(ghub), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_noatom_update, dim3(gw), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PULL_B:
      hipLaunchKernelGGL(k_pull<false>, dim3(std::max(g0, gw)), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PUSH_Q_FILTER: {
      // chunks of the temporary list: F_k's edge total when the host knows it,
      // else every chunk the graph could need (those past the total exit at once)
      int nchunk = cdiv(count, SCAN_CHUNK);
      hipLaunchKernelGGL(k_merge_scan_local, dim3(std::max(g0, clampi(nchunk, 1, GMAX))), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_merge_scan_chunks, dim3(1), dim3(BLOCK), 0, s, a);
      const long long span = dev ? (long long)a.nnz : edges;
      const int chunks = (int)std::max(1ll, (span + a.tmpcap - 1) / a.tmpcap);
      const int ge = clampi(cdiv(std::min(span, (long long)a.tmpcap), MERGE_TILE), 1, GMAX);
      const int gf = clampi(cdiv(std::min(span, (long long)a.tmpcap), BLOCK), 1, GMAX);
      for (int r = 0; r < chunks; ++r) {
        hipLaunchKernelGGL(k_adv_tmp, dim3(ge), dim3(BLOCK), 0, s, a, r);
        hipLaunchKernelGGL(k_filter_tmp, dim3(gf), dim3(BLOCK), 0, s, a, r);
      }
      break;
    }
    case BFS_V_PUSH_B_FILTER: {
      // as PUSH_Q_FILTER, the edge space flattened over bitmap words
      const int nwchunk = cdiv(a.W, SCAN_CHUNK);
      hipLaunchKernelGGL(k_wscan_local, dim3(std::max(g0, clampi(nwchunk, 1, GMAX))), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_wscan_chunks, dim3(1), dim3(BLOCK), 0, s, a);
      const long long span = dev ? (long long)a.nnz : edges;
      const int chunks = (int)std::max(1ll, (span + a.tmpcap - 1) / a.tmpcap);
      const int ge = clampi(cdiv(std::min(span, (long long)a.tmpcap), MERGE_TILE), 1, GMAX);
      const int gf = clampi(cdiv(std::min(span, (long long)a.tmpcap), BLOCK), 1, GMAX);
      for (int r = 0; r < chunks; ++r) {
        hipLaunchKernelGGL(k_adv_tmp_b, dim3(ge), dim3(BLOCK), 0, s, a, r);
        hipLaunchKernelGGL(k_filter_tmp, dim3(gf), dim3(BLOCK), 0, s, a, r);
      }
      break;
    }
    case BFS_V_PUSH_P3:
      hipLaunchKernelGGL(k_push_p3, dim3(std::max(g0, gw)), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_push_hubs<false>, dim3(ghub), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_p3_update, dim3(gw), dim3(BLOCK), 0, s, a);
      break;
    case BFS_V_PULL_VIS:
      hipLaunchKernelGGL(k_pull<true>, dim3(std::max(g0, gw)), dim3(BLOCK), 0, s, a);
      hipLaunchKernelGGL(k_merge_vis, dim3(clampi(cdiv(a.W, BLOCK), 1, GMAX)), dim3(BLOCK), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bfs
