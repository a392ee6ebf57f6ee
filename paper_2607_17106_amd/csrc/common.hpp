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

// Counters of one frontier F_k.  Producers add into one of NSH shards (chosen
// by workgroup id), each on its own 64-byte line: same-address device-scope
// atomics serialise across the XCDs, shards do not.  k_finish reduces the
// shards into the slot's total and the queue segment offsets.
struct alignas(64) LevelCtr {
  u32 count;        // |F_k|: raw reservations in the shard's queue segment
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

constexpr int NSH = 256;  // counter shards / queue segments per level

// One ring slot: NSH producer shards + the overflow queue counter, the
// reduced total, and the queue segment prefix (seg[s] = entries before
// segment s; seg[NSH] = start of the overflow area; seg[NSH+1] = |F_k|).
struct RingSlot {
  LevelCtr sh[NSH + 1];
  LevelCtr tot;
  int seg[NSH + 2];
  int pad[30];
};
static_assert(sizeof(RingSlot) % 256 == 0, "RingSlot must keep 256-byte alignment");

// Per-level log written by k_finish (entry k describes F_k) and loop control.
struct alignas(64) LevelLog {
  u32 count;       // |F_k|
  int variant;     // variant that expanded F_k (device-chosen modes)
  u64 edges, in_edges, ld, ld2;
  u64 scanned;     // edges examined by the step that produced F_k
  int fallback;
  int pad;
  u64 t;           // persistent kernel: device wall clock when F_k was complete
};
static_assert(sizeof(LevelLog) == 64, "LevelLog is one line");
constexpr int LOGCAP = 16384;

struct alignas(64) LoopCtl {
  u64 done;        // 1 once a level produced an empty frontier
  u64 levels;      // number of non-empty levels seen (1 + largest depth)
  u64 reached;     // sum of |F_k|
  u64 comp_edges;  // sum of out-edges of F_k
  u64 pad[4];
};

// Frontier queue: NSH segments of qcap entries, then an overflow area of n.
inline int queue_cap(int n) { return (n + NSH - 1) / NSH; }
inline size_t queue_entries(int n) { return (size_t)queue_cap(n) * NSH + (size_t)n; }
// advance-then-filter: temporary list entries, n clamped to [2^16, 2^22] and
// rounded up to whole merge tiles (chunks of the list start on a tile)
inline int tmp_entries(int n) {
  const int c = n < (1 << 16) ? (1 << 16) : (n > (1 << 22) ? (1 << 22) : n);
  return (c + MERGE_TILE - 1) / MERGE_TILE * MERGE_TILE;
}

// Single-source workspace, carved from one caller buffer.
struct Workspace {
  u64 *vis;            // P: visited bitmap, bits >= n and never-reachable bits pre-set
  u64 *fb[3];          // frontier bitmaps (current, next, dead) rotating by level
  int *q[2];           // frontier queues (current, next), segmented
  int *scan;           // merge path: per-chunk inclusive degree scan
  int *bsum;           // merge path: chunk totals -> exclusive prefix
  int *hubs;           // block variant: deferred high-degree vertices
  RingSlot *ring;      // RING slots
  LevelLog *log;       // LOGCAP entries
  LoopCtl *ctl;
  void *bar;           // grid barrier of the persistent kernel
  int *sched;          // device copy of a host schedule (LOGCAP entries)
  u64 *gsum;           // graph-level sums (ld, ld2), selector state, validation flag
  u64 *vis_prev;       // three-array visited strategy: P_{k-1} (valid while *p3_level == k)
  int *p3_level;
  int *tmp_v, *tmp_u;  // advance-then-filter: temporary list (tmp_entries(n) entries)
  int W;               // bitmap words = ceil(n/64)
  int qcap;
};

size_t workspace_bytes_single(int n);
size_t workspace_bytes_multi(int n);
Workspace carve_single(void *base, int n);

// Arguments of one level step.  k is the level being expanded: vertices it
// discovers get depth k+1.
struct StepArgs {
  int n, W, k, hub, qcap;
  int nnz;                     // edges (bounds the advance-then-filter chunks when F_k's are unknown)
  int gate;                    // -1: always run (host loop); -2: run while F_k is non-empty;
                               // >= 0: run only if F_k is non-empty and its device decision is `gate`
  const int *rp, *ci;          // CSR
  const int *cp, *cx;          // CSC (may alias CSR)
  int *levels, *parents;       // parents may be null
  u64 *vis;
  const u64 *fb_cur;
  u64 *fb_next, *fb_dead;
  const int *q_cur;
  int *q_next;
  LevelCtr *c_cur;             // totals of F_k (consumers add nhub/ntiles/total_e)
  const int *seg_cur;          // queue segment prefix of F_k
  LevelCtr *sh_next;           // shards of F_{k+1} (producers add)
  LevelCtr *sh_zero;           // shards of F_{k+2} (cleared by the first kernel)
  int *scan, *bsum, *hubs;
  u64 *vis_prev;               // PUSH_P3: P_{k-1} when *p3_level == k
  int *p3_level;
  int *tmp_v, *tmp_u;          // PUSH_Q_FILTER: neighbours and their sources
  int tmpcap;                  // their entries (tmp_entries(n))
};

// ------------------------------------------------- per-thread host context
struct HostCtx {
  LevelCtr *pinned = nullptr;  // read-back of one slot total + scratch
  u64 *pinned_u64 = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t lev_ev[64] = {};  // per-level timing in the device loop (2 per level)
  u64 seq = 0;                 // last sequence number a kernel posted to `pinned`
  bool ok = false;
  HostCtx();
};
HostCtx &host_ctx();
// Waits until a kernel on stream s has written `seq` to *flag (pinned host
// memory), polling it; after 2 ms without it, synchronises the stream (which
// reports a failed kernel) and fails if the value is still missing.
int wait_posted(const volatile u64 *flag, u64 seq, hipStream_t s);
// Library-cached device workspace for callers that pass none (one per device).
int cached_workspace(size_t bytes, void **out);

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

// Inclusive 64-bit sum over the wave (every lane active): the DPP steps of
// wave_incl_scan below with two 32-bit moves per step.
__device__ __forceinline__ u64 wave_incl_scan_u64(u64 x) {
#define WAVE_SCAN_STEP(CTRL, ROWS)                                                             \
  {                                                                                            \
    const u32 lo = (u32)__builtin_amdgcn_update_dpp(0, (int)(u32)x, CTRL, ROWS, 0xf, false);   \
    const u32 hi = (u32)__builtin_amdgcn_update_dpp(0, (int)(u32)(x >> 32), CTRL, ROWS, 0xf, false); \
    x += ((u64)hi << 32) | lo;                                                                 \
  }
  WAVE_SCAN_STEP(0x111, 0xf)  // row_shr:1
  WAVE_SCAN_STEP(0x112, 0xf)  // row_shr:2
  WAVE_SCAN_STEP(0x114, 0xf)  // row_shr:4
  WAVE_SCAN_STEP(0x118, 0xf)  // row_shr:8
  WAVE_SCAN_STEP(0x142, 0xa)  // row_bcast:15, rows 1 and 3
  WAVE_SCAN_STEP(0x143, 0xc)  // row_bcast:31, rows 2 and 3
#undef WAVE_SCAN_STEP
  return x;
}

// Sum over the wave (every lane active), returned in every lane: the
// inclusive scan above, then lane 63's total read into every lane.
__device__ __forceinline__ u64 wave_sum_u64(u64 x) {
  x = wave_incl_scan_u64(x);
  const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)x, WAVE - 1);
  const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)(x >> 32), WAVE - 1);
  return ((u64)hi << 32) | lo;
}

// Lane l's value in every lane: a scalar read of one lane (l the same in every
// lane, e.g. derived from a ballot; lane l need not be active now, only have
// written x).
__device__ __forceinline__ u32 lane_bcast(u32 x, int l) { return (u32)__builtin_amdgcn_readlane((int)x, l); }
__device__ __forceinline__ int lane_bcast(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ u64 lane_bcast(u64 x, int l) {
  return ((u64)lane_bcast((u32)(x >> 32), l) << 32) | lane_bcast((u32)x, l);
}
__device__ __forceinline__ float lane_bcast(float x, int l) { return __int_as_float(lane_bcast(__float_as_int(x), l)); }

// OR over the wave (every lane active), in every lane: a DPP inclusive scan
// on each 32-bit half (as wave_incl_scan below), then lane 63's result.
__device__ __forceinline__ u64 wave_or_u64(u64 x) {
  u32 lo = (u32)x, hi = (u32)(x >> 32);
#define WAVE_OR_STEP(CTRL, ROWS)                                            \
  {                                                                         \
    lo |= (u32)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, ROWS, 0xf, false); \
    hi |= (u32)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, ROWS, 0xf, false); \
  }
  WAVE_OR_STEP(0x111, 0xf)  // row_shr:1
  WAVE_OR_STEP(0x112, 0xf)  // row_shr:2
  WAVE_OR_STEP(0x114, 0xf)  // row_shr:4
  WAVE_OR_STEP(0x118, 0xf)  // row_shr:8
  WAVE_OR_STEP(0x142, 0xa)  // row_bcast:15, rows 1 and 3
  WAVE_OR_STEP(0x143, 0xc)  // row_bcast:31, rows 2 and 3
#undef WAVE_OR_STEP
  return ((u64)lane_bcast(hi, WAVE - 1) << 32) | lane_bcast(lo, WAVE - 1);
}

// Maximum over the wave of non-negative ints (every lane active), in every
// lane (a lane with no source in a step takes 0).
__device__ __forceinline__ int wave_max_nonneg(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
  return lane_bcast(x, WAVE - 1);
}

// Inclusive sum over the wave (every lane active).  DPP moves, no LDS: shifts
// by 1, 2, 4 and 8 inside each 16-lane row (a lane with no source adds the
// move's old value, 0), then the last lane of rows 0 and 2 into rows 1 and 3,
// then lane 31 into rows 2 and 3.
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15, rows 1 and 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31, rows 2 and 3
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

// Wave-aggregated append to the counter `*counter` (used for the hub list,
// which stays short).  Works in divergent code.
__device__ __forceinline__ int wave_append(bool pred, u32 *counter) {
  u64 m = __ballot(pred);
  if (m == 0) return -1;
  int leader = __ffsll((long long)m) - 1;
  u32 base = 0;
  if (lane() == leader) base = atomicAdd(counter, (u32)__popcll(m));
  base = lane_bcast(base, leader);
  return pred ? (int)(base + (u32)__popcll(m & __lanemask_lt())) : -1;
}

// Appends v (lanes with pred) to the next frontier queue: one reservation per
// wave in the workgroup's segment; the part that does not fit goes to the
// overflow area.  Works in divergent code.
__device__ __forceinline__ void queue_push(bool pred, int v, const StepArgs &a) {
  const u64 m = __ballot(pred);
  if (m == 0) return;
  const int s = blockIdx.x % NSH;
  const int leader = __ffsll((long long)m) - 1;
  u32 pos = 0;
  if (lane() == leader) pos = atomicAdd(&a.sh_next[s].count, (u32)__popcll(m));
  pos = lane_bcast(pos, leader);
  const int my = (int)pos + __popcll(m & __lanemask_lt());
  const bool over = pred && my >= a.qcap;
  if (pred && !over) a.q_next[(size_t)s * a.qcap + my] = v;
  const u64 mo = __ballot(over);
  if (mo) {
    const int l2 = __ffsll((long long)mo) - 1;
    u32 p2 = 0;
    if (lane() == l2) p2 = atomicAdd(&a.sh_next[NSH].count, (u32)__popcll(mo));
    p2 = lane_bcast(p2, l2);
    if (over) a.q_next[(size_t)NSH * a.qcap + p2 + __popcll(mo & __lanemask_lt())] = v;
  }
}

// Queue position of frontier entry i, given the segment prefix staged in LDS.
__device__ __forceinline__ int queue_slot(const int *seg, int qcap, int i) {
  int lo = 0, hi = NSH;  // last s in [0, NSH] with seg[s] <= i
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seg[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo * qcap + (i - seg[lo]);
}

__device__ __forceinline__ void stage_seg(int *s_seg, const int *seg) {
  for (int i = threadIdx.x; i < NSH + 2; i += BLOCK) s_seg[i] = seg[i];  // BLOCK-wide workgroups
  __syncthreads();
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
  // Must be called by all lanes of the wave (convergent point).  Adds into
  // the workgroup's shard.
  __device__ __forceinline__ void flush(LevelCtr *sh) {
    LevelCtr *c = sh + (blockIdx.x % NSH);
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
// and the counter shards of level k+2.  Called by the first kernel of a step.
__device__ __forceinline__ void clear_dead(const StepArgs &a) {
  const int tid = blockIdx.x * BLOCK + threadIdx.x;  // BLOCK-wide workgroups
  const int nthr = gridDim.x * BLOCK;
  for (int i = tid; i < a.W; i += nthr) a.fb_dead[i] = 0ull;
  u32 *z = reinterpret_cast<u32 *>(a.sh_zero);
  const int nz = (NSH + 1) * (int)(sizeof(LevelCtr) / sizeof(u32));
  for (int i = tid; i < nz; i += nthr) z[i] = 0u;
}

// Device-loop gate: true when this launch should not run level k (another
// variant was chosen, or the search has finished).  Uniform per kernel.
__device__ __forceinline__ bool gated_off(const StepArgs &a) {
  if (a.gate == -1) return false;
  if (a.c_cur->count == 0u) return true;
  return a.gate >= 0 && a.c_cur->decision != a.gate;
}

// ---------------------------------------------------------------- launch
// Launchers (defined in the .hip files).  All enqueue on `s`.
// k_reset (clears the state and the ring) and, with f0, k_reset_f0 (F_0 = {src} in slot 0).
hipError_t launch_reset(const StepArgs &a, int src, RingSlot *ring, hipStream_t s, bool f0 = true);
// count < 0: sizes unknown on the host (device loop); fixed grids are used.
hipError_t launch_step(int variant, const StepArgs &a, int count, long long edges, hipStream_t s);
hipError_t launch_finish(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl, hipStream_t s);
hipError_t launch_state_from_depths(const StepArgs &a, const int *depths, RingSlot *ring, hipStream_t s);
hipError_t launch_graph_ld(int n, const int *rp, u64 *gsum, hipStream_t s);
hipError_t launch_validate(int n, int nnz, const int *ptr, const int *idx, u64 *flag, hipStream_t s);
// Checks offsets and ids of the CSR (and CSC); BFS_EGRAPH if malformed.  Synchronises.
int validate_graph(const bfs_graph *g, u64 *flag_dev, hipStream_t s);
int min_first_grid(int W);

}  // namespace bfs
