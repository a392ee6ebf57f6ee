// Shared device helpers and host-side plumbing of the BFS library (gfx950,
// wave64).  Nothing here is public; the C ABI is include/bfs_eeds.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "../../include/bfs_eeds.h"

namespace bfs {

typedef unsigned long long u64;
typedef unsigned int u32;

constexpr int WAVE = 64;
constexpr int BLOCK = 256;               // 4 waves per workgroup
constexpr int RING = 4;                  // per-level counter slots in flight
constexpr int SCAN_CHUNK = 1024;         // merge path: entries per scan block
constexpr int MERGE_TILE = 2048;         // merge path: edges per tile
constexpr int MERGE_STAGE = 2304;        // merge path: frontier entries staged per tile
constexpr int DEFAULT_HUB = 2048;        // block variant: degree above which a vertex is split grid-wide

// Counters of one frontier F_k, accumulated by the step that produced it.
struct alignas(64) LevelCtr {
  u32 count;        // |F_k| (also the queue length)
  u32 nhub;         // block variant: hub list length while F_k is expanded
  u64 edges;        // sum over F_k of out-degree
  u64 in_edges;     // sum over F_k of in-degree
  u64 ld;           // sum over F_k of floor(log2(1+outdeg))
  u64 ld2;          // sum of its squares
  u64 scanned;      // edges examined by the step that produced F_k
  u32 ntiles;       // merge path: tiles while F_k is expanded
  u32 total_e;      // merge path: scanned total of F_k's degrees
  int decision;     // device-side choice of the variant that expands F_k
  int fallback;     // 1 when the learned selector deferred to the heuristic
};
static_assert(sizeof(LevelCtr) == 64, "LevelCtr must stay one 64-byte line");

// Single-source workspace, carved from one caller buffer.
struct Workspace {
  u64 *vis;            // P: visited bitmap, bits >= n pre-set
  u64 *fb[3];          // frontier bitmaps (current, next, dead) rotating by level
  int *q[2];           // frontier queues (current, next)
  int *scan;           // merge path: per-chunk inclusive degree scan
  int *bsum;           // merge path: chunk totals -> exclusive prefix
  int *hubs;           // block variant: deferred high-degree vertices
  LevelCtr *ctr;       // RING slots
  u64 *gsum;           // graph-level sums (ld, ld2) and validation flag
  int W;               // bitmap words = ceil(n/64)
};

size_t workspace_bytes_single(int n);
size_t workspace_bytes_multi(int n);
Workspace carve_single(void *base, int n);

// Arguments of one level step.  k is the level being expanded: vertices it
// discovers get depth k+1.
struct StepArgs {
  int n, W, k, hub;
  const int *rp, *ci;          // CSR
  const int *cp, *cx;          // CSC (may alias CSR)
  int *levels, *parents;       // parents may be null
  u64 *vis;
  const u64 *fb_cur;
  u64 *fb_next, *fb_dead;
  const int *q_cur;
  int *q_next;
  LevelCtr *c_cur, *c_next, *c_zero;
  int *scan, *bsum, *hubs;
};

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
#define BFS_HIP(call)                                                  \
  do {                                                                 \
    hipError_t _e = (call);                                            \
    if (_e != hipSuccess) return ::bfs::hip_fail(_e, #call);           \
  } while (0)

// ------------------------------------------------------- device helpers
__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ u64 wave_sum_u64(u64 x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int l = lane();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int y = __shfl_up(x, (unsigned)o);
    if (l >= o) x += y;
  }
  return x;
}

// Exclusive scan over a BLOCK-thread workgroup; *total gets the sum.
// s_w must hold BLOCK/WAVE ints.  Contains two barriers.
__device__ __forceinline__ int block_excl_scan(int x, int *total, int *s_w) {
  const int w = threadIdx.x / WAVE;
  int incl = wave_incl_scan(x);
  if (lane() == WAVE - 1) s_w[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / WAVE; ++i) {
    int t = s_w[i];
    off += (i < w) ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

// Wave-aggregated append: lanes with pred get consecutive slots from one
// atomicAdd on *counter; returns the slot or -1.  Works in divergent code
// (only the lanes active at the call take part).
__device__ __forceinline__ int wave_append(bool pred, u32 *counter) {
  u64 m = __ballot(pred);
  if (m == 0) return -1;
  int leader = __ffsll((long long)m) - 1;
  u32 base = 0;
  if (lane() == leader) base = atomicAdd(counter, (u32)__popcll(m));
  base = __shfl(base, leader);
  return pred ? (int)(base + (u32)__popcll(m & __lanemask_lt())) : -1;
}

__device__ __forceinline__ bool test_bit(const u64 *bm, int v) {
  return (bm[v >> 6] >> (v & 63)) & 1ull;
}

// floor(log2(1 + d)) for d >= 0
__device__ __host__ __forceinline__ int ilog2p1(int d) {
#ifdef __HIP_DEVICE_COMPILE__
  return 31 - __clz((unsigned)d + 1u);
#else
  return 31 - __builtin_clz((unsigned)d + 1u);
#endif
}

// Per-lane accumulators of new-vertex statistics, reduced once per wave.
struct NewStats {
  u64 edges = 0, in_edges = 0, ld = 0, ld2 = 0, scanned = 0;
  __device__ __forceinline__ void add_vertex(const StepArgs &a, int v) {
    int d = a.rp[v + 1] - a.rp[v];
    int di = (a.cp == a.rp) ? d : (a.cp ? a.cp[v + 1] - a.cp[v] : d);
    int l = ilog2p1(d);
    edges += (u64)d;
    in_edges += (u64)di;
    ld += (u64)l;
    ld2 += (u64)(l * l);
  }
  // Must be called by all lanes of the wave (convergent point).
  __device__ __forceinline__ void flush(LevelCtr *c) {
    u64 e = wave_sum_u64(edges), ie = wave_sum_u64(in_edges), a = wave_sum_u64(ld),
        b = wave_sum_u64(ld2), s = wave_sum_u64(scanned);
    if (lane() == 0) {
      if (e) atomicAdd(&c->edges, e);
      if (ie) atomicAdd(&c->in_edges, ie);
      if (a) atomicAdd(&c->ld, a);
      if (b) atomicAdd(&c->ld2, b);
      if (s) atomicAdd(&c->scanned, s);
    }
  }
};

// Zeroes the dead frontier bitmap (it receives F_{k+2} at the next level)
// and the counter slot of level k+2.  Called by the first kernel of a step.
__device__ __forceinline__ void clear_dead(const StepArgs &a) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthr = gridDim.x * blockDim.x;
  for (int i = tid; i < a.W; i += nthr) a.fb_dead[i] = 0ull;
  if (tid < (int)(sizeof(LevelCtr) / sizeof(u32))) reinterpret_cast<u32 *>(a.c_zero)[tid] = 0u;
}

// ---------------------------------------------------------------- launch
// Launchers (defined in the .hip files).  All enqueue on `s`.
hipError_t launch_reset(const StepArgs &a, int src, hipStream_t s);
hipError_t launch_step(int variant, const StepArgs &a, int count, long long edges, hipStream_t s);
hipError_t launch_state_from_depths(const StepArgs &a, const int *depths, hipStream_t s);
hipError_t launch_graph_ld(int n, const int *rp, u64 *gsum, hipStream_t s);
hipError_t launch_validate(int n, int nnz, const int *ptr, const int *idx, u64 *flag, hipStream_t s);
int min_first_grid(int W);

}  // namespace bfs
