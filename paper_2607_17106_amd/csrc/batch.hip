// Batched BFS: many independent graphs (a disjoint union stored back to
// back) searched in one persistent launch.
//
// The host orders the instances largest first and gives each a team size:
// an instance small enough for LDS (n <= small_vertices) is one task, run by
// one workgroup alone; a larger one is G tasks (G from team_vertices and
// max_team), one per member of a team of workgroups that search it together.
// Every workgroup repeatedly takes the next task from a ticket counter, so the
// members of a team start together (their tickets are consecutive) and the
// launch drains as a whole.  Each level is Cascade 1's step
// (F_{k+1} = N(F_k) AND NOT P_k, P_{k+1} = P_k OR F_{k+1}).
//
// Single workgroup (n <= small_vertices): the visited bitmap lives in LDS
// (gfx950's 160 KB hold it for 2^20 vertices), so every claim is an LDS
// atomic; device-wide 64-bit atomics run at about 27 G/s on this chip, loads
// at ten times that, so a per-edge global atomic would bound the batch.  The
// frontier is a queue in the instance's global state (each entry the vertex
// with its row offsets), and all synchronisation is workgroup barriers.
//   top-down: 2 x block_threads queue vertices per pass.  A list of at most
//     LIGHT edges is expanded by its vertex's own lane in rounds of 4 edges
//     (the lane's 2 vertices at once), each wave on its own; the winners of
//     unvisited targets' LDS atomicOr are staged per wave in LDS and recorded
//     64 at a time (depth, row offsets, queue entry; one reservation per
//     flush).  On levels with longer lists a second sweep flattens them with a
//     workgroup scan (Table 3, variant 1 at workgroup scale), each lane taking
//     U consecutive edges per round.
//   bottom-up (symmetric instances): the queue is scattered into a frontier
//     bitmap (LDS when it fits, else global); each wave owns 64 consecutive
//     vertices, tests the first in-edges of every unvisited one (loads issued
//     together) and scans the rest wave-cooperatively, stopping at the first
//     frontier member.
//
// Teams (larger instances): G co-resident workgroups search the instance
// together.  Each vertex has a stamp byte (0 unvisited, else 1 + depth mod
// 255) in the team's state, and the vertices are dealt to the members in
// interleaved 16384-vertex chunks.  No atomics touch the search state: every
// access to a stamp is a device-scope load or store, and a stamp or depth
// written by two members at one level is written twice with the same value
// (the paper's atomic-free update, Table 3, variants 21 and 24).  Per level:
//   top-down: each member reads its frontier off its own vertices' stamps
//     (owner computes), lists it in LDS, and expands it as the single
//     workgroup does, stamping and recording every unvisited target.
//   bottom-up: each member handles its own unvisited vertices, reading the
//     in-neighbours' stamps.
// A level ends at a team barrier: each member publishes its counts (vertices
// found, their out-edges), waits until all G members have arrived on the
// team's counter, then sums every member's counts in the same order, so all
// members take the same direction for the next level and stop together.
// 64-bit atomics run at about 27 G/s on this chip against ten times that for
// loads, so the team path avoids them on the search state; device-scope
// accesses are coherent across the XCDs' L2 caches without the writeback and
// invalidate a device-scope fence costs, and before arriving each wave waits
// for its own stores to complete.  Every wait is bounded: a member whose wait
// runs out raises the team's abort flag, every member leaves, and the call
// reports an error.  Teams never exceed the grid, and the grid never exceeds
// what can be resident at once, so every member of a team runs.
// Depths: the single workgroup writes each depth once; a team writes a
// reached vertex's depth once per finder (same value) and the -1 of an
// unreached vertex at the end, from its owner.
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace bfs {

constexpr int MAX_TEAM = 16;            // members per team (bfs_batch_config.max_team <= this)
constexpr int LIGHT = 8;                // top-down: out-degree up to which a lane expands its own vertex
constexpr int BATCH_T = 4;              // bottom-up: in-edges each lane tests before the wave-cooperative scan
constexpr unsigned long long WAIT_TICKS = 200000000ull;  // team barrier wait bound: 2 s of the 100 MHz clock

// Team control block (one per team instance, at the start of its state).
struct TeamCtl {
  u32 arrive;                // barrier arrivals, monotonic: the g-th barrier completes at g * G
  u32 abort;                 // set when a member's wait timed out
  u32 pad[14];
  u64 slot[2][MAX_TEAM][2];  // per level parity and member: vertices found, their out-edges
};
constexpr size_t TEAM_CTL_BYTES = 1024;
static_assert(sizeof(TeamCtl) <= TEAM_CTL_BYTES, "team control block");

struct BatchArgs {
  int num, ntask;
  const int *v_off;         // [num+1]
  const int *task;          // [ntask][2]: instance, member (-1: single workgroup, LDS bitmaps)
  const int *team_g;        // [num] team size (0 for single-workgroup instances)
  const long long *toff;    // [num] byte offset of the instance's team state
  const int *src;           // [num] local sources
  const int *rp;            // concatenated CSR: global entry offsets
  const int *ci;            // local column ids
  int *levels;              // [total_n]
  u64 *stats;               // [num][2]: component out-edges, levels
  int *ticket;
  int *err;                 // 1 when a team barrier timed out
  char *team;               // per-instance states (single-workgroup and team instances)
  int small_n;              // one workgroup, visited bitmap in LDS, when n <= small_n
  int fr_lds;               // 1: the bottom-up frontier bitmap fits in LDS beside the visited bitmap
  int symmetric;
  int nnz;                  // entries of col_idx (bounds the 16-byte list reads)
};

// ------------------------------------------------------------ helpers
__device__ __forceinline__ u64 or_wg(u64 *p, u64 bits) {
  return __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Frontier-bitmap test: an atomic load at workgroup scope, so it observes the
// workgroup's atomic ORs that precede the last barrier.
__device__ __forceinline__ bool in_frontier(u64 *fr, int u) {
  return (__hip_atomic_load(fr + (u >> 6), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> (u & 63)) & 1ull;
}
// Device-scope relaxed atomics: the only accesses to state shared by a team.
__device__ __forceinline__ u64 ld_dev(u64 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 ld_dev32(u32 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(u64 *p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// rp[u] and rp[u+1] with one 8-byte load (dword-aligned wide loads are legal
// on this chip): one memory request per list instead of two.
__device__ __forceinline__ int2 rp_pair(const int *rp, int u) {
  int2 r;
  __builtin_memcpy(&r, rp + u, 8);
  return r;
}
// Entries t0 .. t0+3 of the list [bg, bg + d) (-1 past its end) with one
// 16-byte load when the four entries lie inside col_idx (nnz entries).
__device__ __forceinline__ void list4(const int *ci, int bg, int d, int t0, int nnz, int *v) {
  if (t0 < d && bg + t0 + 4 <= nnz) {
    int4 x;
    __builtin_memcpy(&x, ci + bg + t0, 16);
    v[0] = x.x;
    v[1] = t0 + 1 < d ? x.y : -1;
    v[2] = t0 + 2 < d ? x.z : -1;
    v[3] = t0 + 3 < d ? x.w : -1;
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = t0 + t < d ? ci[bg + t0 + t] : -1;
  }
}

// Last index i in [0, cap) with incl[i] > e (incl ascending, incl[cap-1] > e).
__device__ __forceinline__ int owner_of(const int *incl, int cap, int e) {
  int lo = 0, hi = cap - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (incl[mid] > e) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Bottom-up direction test shared by both forms.  One searcher pays for every
// in-edge a bottom-up step reads.  An unvisited vertex reads about
// (e_U + e_F) / e_F in-edges before it meets a frontier member (in-edges drawn
// at random), and at most its degree, so the step reads about
// min(e_U, n_U (e_U + e_F) / e_F); the top-down step reads e_F.
__device__ __forceinline__ int choose_bottom_up(long long nU, long long eU, long long eF) {
  const long long scan = eF > 0 ? min(eU, nU * ((eU + eF) / eF + 1)) : eU;
  return scan < eF ? 1 : 0;
}

// ------------------------------------------- single workgroup, LDS visited
// Per-instance state in global memory: two frontier queues (n entries each)
// and, when it does not fit in LDS beside the visited bitmap, the bottom-up
// frontier bitmap.  Only this workgroup touches them, so plain accesses are
// coherent.  A queue entry is the vertex with its row offsets (three int
// arrays), read when its finder records it: expanding it then reads the entry
// with coalesced loads instead of a second scattered rp access.
struct SQueue {
  int *v, *b, *e;  // vertex, rp[v], rp[v + 1]
};
__host__ __device__ inline size_t single_state_bytes(long long n, bool fr_global) {
  const size_t qb = ((size_t)n * 4 + 255) & ~(size_t)255;
  const size_t wb = ((size_t)((n + 63) / 64) * 8 + 255) & ~(size_t)255;
  return 6 * qb + (fr_global ? wb : 0);
}

// Appends the candidates of one round (won[j] per lane) to q at slots taken
// from the LDS counter *cnt with one reservation per wave; records depth k+1
// and the new vertices' out-edges.  Called by every lane of the wave.
template <int U>
__device__ __forceinline__ void single_found(const int *rp, int *lv, const bool *won, const int *v, int k,
                                             const SQueue &q, int *cnt, u64 &efn) {
  u64 mk[U];
  int tot = 0;
#pragma unroll
  for (int j = 0; j < U; ++j) {
    if (won[j]) lv[v[j]] = k + 1;
    mk[j] = __ballot(won[j]);
    tot += __popcll(mk[j]);
  }
  if (!tot) return;
  int2 r[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    r[j] = make_int2(0, 0);
    if (won[j]) r[j] = rp_pair(rp, v[j]);
  }
  int base = 0;
  if (lane() == 0) base = atomicAdd(cnt, tot);
  base = lane_bcast(base, 0);
#pragma unroll
  for (int j = 0; j < U; ++j) {
    if (won[j]) {
      const int slot = base + __popcll(mk[j] & __lanemask_lt());
      q.v[slot] = v[j];
      q.b[slot] = r[j].x;
      q.e[slot] = r[j].y;
      efn += (u64)(r[j].y - r[j].x);
    }
    base += __popcll(mk[j]);
  }
}

// Light top-down rounds stage their finds per wave in LDS (STAGE vertices per
// wave), so that recording them takes dense wave instructions: a lane's 16
// candidates are found by few lanes each, and a per-candidate masked store or
// load costs the texture unit about as much as a full one.
constexpr int STAGE = 256;

// Records the wave's staged finds stg[0, cnt) (cnt <= STAGE): depth k+1 and
// queue entries with their row offsets, one queue reservation, 64 per round.
// Called by every lane of the wave.
__device__ __forceinline__ void stage_flush(const int *rp, int *lv, const int *stg, int cnt, int k, const SQueue &q,
                                            int *qcnt, u64 &efn) {
  if (cnt == 0) return;  // uniform per wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int base = 0;
  if (lane() == 0) base = atomicAdd(qcnt, cnt);
  base = lane_bcast(base, 0);
  constexpr int R = STAGE / WAVE;
  int w[R];
  int2 r[R];
#pragma unroll
  for (int o = 0; o < R; ++o) {
    const int i = o * WAVE + lane();
    w[o] = i < cnt ? stg[i] : -1;
  }
#pragma unroll
  for (int o = 0; o < R; ++o) r[o] = w[o] >= 0 ? rp_pair(rp, w[o]) : make_int2(0, 0);
#pragma unroll
  for (int o = 0; o < R; ++o) {
    if (w[o] < 0) continue;
    const int slot = base + o * WAVE + lane();
    lv[w[o]] = k + 1;
    q.v[slot] = w[o];
    q.b[slot] = r[o].x;
    q.e[slot] = r[o].y;
    efn += (u64)(r[o].y - r[o].x);
  }
  // the stage is written again only after every lane has read it
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds the wave's finds of one group of G candidates per lane (won[j]) to the
// stage, first flushing it when they would not fit (G * WAVE <= STAGE).
template <int G>
__device__ __forceinline__ void stage_add(const int *rp, int *lv, int *stg, int &scnt, const bool *won, const int *v,
                                          int k, const SQueue &q, int *qcnt, u64 &efn) {
  static_assert(G * WAVE <= STAGE, "a group fits the stage");
  u64 mk[G];
  int gt = 0;
#pragma unroll
  for (int j = 0; j < G; ++j) {
    mk[j] = __ballot(won[j]);
    gt += __popcll(mk[j]);
  }
  if (gt == 0) return;  // uniform per wave
  if (scnt + gt > STAGE) {
    stage_flush(rp, lv, stg, scnt, k, q, qcnt, efn);
    scnt = 0;
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    if (won[j]) stg[scnt + __popcll(mk[j] & __lanemask_lt())] = v[j];
    scnt += __popcll(mk[j]);
  }
}

template <int BT>
__device__ void search_single(const BatchArgs &A, int b, char *dyn, int *s_off, int *s_incl, int *s_w, int *s_qn,
                              unsigned long long *s_efn) {
  // queue vertices per lane per pass: 2 keeps the 1024-thread form within its
  // 128 registers with less spilling than 4 (20 bytes a lane against 60;
  // a side-1024 lattice 4.6 -> 4.45 ms).  Even: the long-list sweep takes a
  // lane's vertices in pairs.
  constexpr int VPT = 2;
  constexpr int CAP = VPT * BT;      // queue vertices per pass
  constexpr int HCAP = 2 * BT;       // heavy lists flattened per half pass
  constexpr int U = 4;               // heavy edges per lane per round
  const int wv = threadIdx.x / WAVE, nwv = BT / WAVE;
  static_assert(4 * BT >= STAGE * (BT / WAVE), "s_off and s_incl hold every wave's stage");
  int *stg = s_off + wv * STAGE;  // this wave's stage: s_off and s_incl are contiguous (light rounds only)
  const int V0 = A.v_off[b];
  const int n = A.v_off[b + 1] - V0;
  const int *rp = A.rp + V0;
  int *lv = A.levels + V0;
  const int W = (n + 63) / 64;
  char *st = A.team + A.toff[b];
  const size_t qb = ((size_t)n * 4 + 255) & ~(size_t)255;
  SQueue qc = {reinterpret_cast<int *>(st), reinterpret_cast<int *>(st + qb), reinterpret_cast<int *>(st + 2 * qb)};
  SQueue qn = {reinterpret_cast<int *>(st + 3 * qb), reinterpret_cast<int *>(st + 4 * qb),
               reinterpret_cast<int *>(st + 5 * qb)};
  u64 *vis = reinterpret_cast<u64 *>(dyn);
  u64 *fr = A.fr_lds ? vis + (A.small_n + 63) / 64 : reinterpret_cast<u64 *>(st + 6 * qb);
  const int src = A.src[b];
  for (int v = threadIdx.x; v < n; v += BT) lv[v] = (v == src) ? 0 : -1;
  for (int w = threadIdx.x; w < W; w += BT) {
    u64 x = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    if (w == W - 1 && (n & 63)) x |= ~0ull << (n & 63);
    vis[w] = x;
  }
  if (threadIdx.x == 0) {
    const int2 r = rp_pair(rp, src);
    qc.v[0] = src;
    qc.b[0] = r.x;
    qc.e[0] = r.y;
    *s_qn = 1;
    *s_efn = (unsigned long long)(r.y - r.x);
  }
  __syncthreads();
  long long nF = *s_qn, eF = (long long)*s_efn;
  long long eU = (long long)(rp[n] - rp[0]) - eF;
  long long nU = n - 1;
  long long comp = eF;
  int k = 0;
  for (;; ++k) {
    const int dir = A.symmetric ? choose_bottom_up(nU, eU, eF) : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      *s_qn = 0;
      *s_efn = 0ull;
    }
    __syncthreads();
    u64 efn = 0;  // out-edges of the vertices this lane discovers (reduced per wave below)
    if (dir == 0) {
      // ---- top-down, CAP queue vertices per pass: lists of out-degree <= LIGHT
      // expanded by their own lane in rounds of 4 edges (no search), every
      // wave on its own (no barrier between passes); then, if the level has
      // longer lists, a second sweep flattens them over the workgroup (U
      // consecutive edges per lane per round, one owner search then a linear
      // walk); claims are LDS atomics
      bool lheavy = false;
      for (int p0 = 0; p0 < nF; p0 += CAP) {
        int beg[VPT], dd[VPT];
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
          const int i = p0 + r * BT + (int)threadIdx.x;
          beg[r] = dd[r] = 0;
          if (i < nF) {
            beg[r] = qc.b[i];
            dd[r] = qc.e[i] - beg[r];
          }
          lheavy |= dd[r] > LIGHT;
        }
        int lmax = 0;
#pragma unroll
        for (int r = 0; r < VPT; ++r)
          if (dd[r] <= LIGHT) lmax = max(lmax, dd[r]);
        lmax = wave_max_nonneg(lmax);
        int scnt = 0;  // staged finds of this wave (stg)
        for (int t0 = 0; t0 < lmax; t0 += 4) {
          int v[4 * VPT];
          bool won[4 * VPT];
#pragma unroll
          for (int r = 0; r < VPT; ++r) list4(A.ci, beg[r], dd[r] <= LIGHT ? dd[r] : 0, t0, A.nnz, v + 4 * r);
#pragma unroll
          for (int j = 0; j < 4 * VPT; ++j) {
            won[j] = false;
            if (v[j] >= 0) {
              const u64 bit = 1ull << (v[j] & 63);
              if (!(vis[v[j] >> 6] & bit)) won[j] = !(or_wg(vis + (v[j] >> 6), bit) & bit);
            }
          }
#pragma unroll
          for (int r = 0; r < VPT; ++r) stage_add<4>(rp, lv, stg, scnt, won + 4 * r, v + 4 * r, k, qn, s_qn, efn);
        }
        stage_flush(rp, lv, stg, scnt, k, qn, s_qn, efn);
      }
      // (the barrier also ends every wave's use of its stage: the heavy sweep
      // writes s_off and s_incl)
      const bool any_heavy = __syncthreads_or(lheavy);
      for (int p0 = 0; any_heavy && p0 < nF; p0 += CAP) {  // uniform per workgroup
        int beg[VPT], dd[VPT];
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
          const int i = p0 + r * BT + (int)threadIdx.x;
          beg[r] = dd[r] = 0;
          if (i < nF) {
            beg[r] = qc.b[i];
            dd[r] = qc.e[i] - beg[r];
          }
        }
        // heavy lists, two halves of the pass (HCAP list entries each)
        bool heavy = false;
#pragma unroll
        for (int r = 0; r < VPT; ++r) heavy |= dd[r] > LIGHT;
        if (!__syncthreads_or(heavy)) continue;
#pragma unroll
        for (int h = 0; h < VPT / 2; ++h) {
          int run = 0, deg[2];
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const int d = dd[2 * h + r];
            run += d > LIGHT ? d : 0;
            deg[r] = run;
          }
          int etot;
          const int eoff = bscan_excl<BT>(run, &etot, s_w);
          if (etot == 0) continue;  // uniform: the workgroup total
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const int i = threadIdx.x * 2 + r;
            const int inc = eoff + deg[r];
            const int d = deg[r] - (r ? deg[r - 1] : 0);
            s_incl[i] = inc;
            s_off[i] = beg[2 * h + r] - (inc - d);
          }
          __syncthreads();
          for (int e0 = (int)threadIdx.x * U; e0 - (int)threadIdx.x * U < etot; e0 += BT * U) {
            int v[U];
            bool won[U];
            int o = e0 < etot ? owner_of(s_incl, HCAP, e0) : 0;
#pragma unroll
            for (int j = 0; j < U; ++j) {
              const int e = e0 + j;
              v[j] = -1;
              if (e < etot) {
                while (s_incl[o] <= e) ++o;
                v[j] = A.ci[s_off[o] + e];
              }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
              won[j] = false;
              if (v[j] >= 0) {
                const u64 bit = 1ull << (v[j] & 63);
                if (!(vis[v[j] >> 6] & bit)) won[j] = !(or_wg(vis + (v[j] >> 6), bit) & bit);
              }
            }
            single_found<U>(rp, lv, won, v, k, qn, s_qn, efn);
          }
          __syncthreads();
        }
      }
    } else {
      // ---- bottom-up: frontier bitmap from the queue, then one wave per word
      for (int w = threadIdx.x; w < W; w += BT) fr[w] = 0ull;
      __syncthreads();
      for (int i = threadIdx.x; i < nF; i += BT) {
        const int u = qc.v[i];
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
          int u[BATCH_T];
#pragma unroll
          for (int t2 = 0; t2 < BATCH_T; ++t2) u[t2] = t2 < d ? A.ci[bb + t2] : -1;
#pragma unroll
          for (int t2 = 0; t2 < BATCH_T; ++t2) found = found || (u[t2] >= 0 && in_frontier(fr, u[t2]));
          pending = !found && d > BATCH_T;
          bb += BATCH_T;
        }
        u64 pm = __ballot(pending);
        while (pm) {
          const int l = __ffsll((long long)pm) - 1;
          pm &= pm - 1;
          const int vb = lane_bcast(bb, l), ve = lane_bcast(ee, l);
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
          if (lane() == 0) vis[w] = vw | m;  // this wave owns word w
          single_found<1>(rp, lv, &found, &v, k, qn, s_qn, efn);
        }
      }
    }
    {
      const u64 we = wave_sum_u64(efn);
      if (lane() == 0 && we) atomicAdd(s_efn, (unsigned long long)we);
    }
    __syncthreads();
    nF = *s_qn;
    eF = (long long)*s_efn;
    eU -= eF;  // symmetric instances: in-edges = out-edges of the new vertices
    nU -= nF;
    comp += eF;
    const SQueue tq = qc;
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

// --------------------------------------------------------------- teams
// Team state: control block | stamp bytes st[n] (zeroed before the launch).
// st[v] = 0 while v is unvisited, else 1 + depth(v) mod 255.  A stamp is
// written with the same value by any member that finds v at that level (no
// atomics: the paper's atomic-free update, Table 3, variant 21, with the
// owner-computes frontier of variant 24: each member reads the next frontier
// off its own vertices' stamps).  Stamps repeat every 255 levels: a vertex 255
// levels older than the frontier also matches it, and expanding it again finds
// only visited neighbours (they are at most one level deeper than it), while a
// bottom-up vertex adjacent to it is visited already; so depths stay exact.
__host__ __device__ inline size_t team_state_bytes(long long n) {
  return TEAM_CTL_BYTES + (((size_t)n + 255) & ~(size_t)255);
}
__device__ __forceinline__ unsigned stamp_of(int depth) { return 1u + (unsigned)(depth % 255); }

typedef unsigned char u8;
__device__ __forceinline__ unsigned ld_st(u8 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_st(u8 *p, unsigned v) {
  __hip_atomic_store(p, (u8)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Member m owns the 16384-vertex chunks m, m + G, ...; `seg` counts its
// 16-vertex segments in order.  Returns the segment's first vertex.
constexpr int TEAM_CV = 16384;
__device__ __forceinline__ int team_seg(int m, int G, int seg) {
  constexpr int SPC = TEAM_CV / 16;
  return (m + G * (seg / SPC)) * TEAM_CV + (seg % SPC) * 16;
}
// Number of segments in member m's chunks (the last chunk cut at n).
__device__ __forceinline__ int team_nseg(int m, int G, int n) {
  const int nch = (n + TEAM_CV - 1) / TEAM_CV;
  if (m >= nch) return 0;
  const int mine = (nch - 1 - m) / G + 1;
  const int last = m + G * (mine - 1);
  return (mine - 1) * (TEAM_CV / 16) + (min(TEAM_CV, n - last * TEAM_CV) + 15) / 16;
}

// Team barrier number `gen` (1, 2, ...): every member arrives once per
// barrier.  Returns false in every thread when the team aborted.
template <int BT>
__device__ bool team_barrier(TeamCtl *c, int G, u32 gen, int *s_flag, int *err) {
  // this wave's device-scope stores are complete before arriving
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    if (G > 1) {
      __hip_atomic_fetch_add(&c->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const u32 target = gen * (u32)G;
      const unsigned long long t0 = wall_clock64();
      while (ld_dev32(&c->arrive) < target) {
        if (ld_dev32(&c->abort) != 0u) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > WAIT_TICKS) {
          __hip_atomic_store(&c->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    } else if (ld_dev32(&c->abort) != 0u) {
      ok = 0;
    }
    *s_flag = ok;
  }
  __syncthreads();
  const bool ok = *s_flag != 0;
  __syncthreads();
  return ok;
}

// One round of top-down candidates (v[j] >= 0): a target whose stamp is 0 is
// stamped for depth k+1 and its depth written; a target found by two lanes in
// the same level is written twice with the same values, and counted twice
// (the counts only steer the direction rule and the stop test).
template <int U>
__device__ __forceinline__ void team_visit(u8 *st, const int *rp, int *lv, const int *v, int k, u32 &cnt, u64 &efn) {
  unsigned sv[U];
#pragma unroll
  for (int j = 0; j < U; ++j) sv[j] = v[j] >= 0 ? ld_st(st + v[j]) : 1u;
  const unsigned nxt = stamp_of(k + 1);
  int d[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    d[j] = 0;
    if (sv[j] == 0u) {
      put_st(st + v[j], nxt);
      lv[v[j]] = k + 1;
      const int2 r = rp_pair(rp, v[j]);
      d[j] = r.y - r.x;
    }
  }
#pragma unroll
  for (int j = 0; j < U; ++j)
    if (sv[j] == 0u) {
      ++cnt;
      efn += (u64)d[j];
    }
}

template <int BT>
__device__ void search_team(const BatchArgs &A, int b, int m, char *dyn, int *s_off, int *s_incl, int *s_w,
                            int *s_flag, u32 *s_cnt, unsigned long long *s_efn) {
  constexpr int VPT = 4;             // listed frontier vertices per lane per pass
  constexpr int LCAP = VPT * BT;     // frontier list entries (LDS)
  constexpr int HCAP = 2 * BT;       // heavy lists flattened per half pass
  constexpr int U = 4;               // heavy edges per lane per round
  constexpr int SG = 8;              // 16-vertex segments scanned per lane per group
  const int wv = threadIdx.x / WAVE, nwv = BT / WAVE;
  int *s_list = reinterpret_cast<int *>(dyn);
  const int G = A.team_g[b];
  const int V0 = A.v_off[b];
  const int n = A.v_off[b + 1] - V0;
  const int *rp = A.rp + V0;
  int *lv = A.levels + V0;
  const int src = A.src[b];
  TeamCtl *ctl = reinterpret_cast<TeamCtl *>(A.team + A.toff[b]);
  u8 *st = reinterpret_cast<u8 *>(A.team + A.toff[b] + TEAM_CTL_BYTES);
  const int nseg = team_nseg(m, G, n);
  const int dsrc = rp[src + 1] - rp[src];
  if (m == 0 && threadIdx.x == 0) {
    lv[src] = 0;
    put_st(st + src, stamp_of(0));
  }
  u32 gen = 1;
  if (!team_barrier<BT>(ctl, G, gen++, s_flag, A.err)) return;
  long long nF = 1, eF = dsrc;
  long long eU = (long long)(rp[n] - rp[0]) - eF;
  long long nU = n - 1;
  int k = 0;
  for (;; ++k) {
    const int dir = A.symmetric ? choose_bottom_up(nU, eU, eF) : 0;
    if (threadIdx.x == 0) {
      *s_cnt = 0u;
      *s_efn = 0ull;
    }
    __syncthreads();
    u32 cnt = 0;
    u64 efn = 0;
    const unsigned cur = stamp_of(k);
    if (dir == 0) {
      // ---- top-down: read my frontier off the stamps, SG segments per lane
      // per group, list it in LDS, expand it
      for (int g0 = 0; g0 < nseg; g0 += SG * BT) {
        u64 w[SG][2];
#pragma unroll
        for (int j = 0; j < SG; ++j) {
          const int sg = g0 + j * BT + (int)threadIdx.x;
          if (sg < nseg) {
            u64 *p = reinterpret_cast<u64 *>(st + team_seg(m, G, sg));
            w[j][0] = ld_dev(p);
            w[j][1] = ld_dev(p + 1);
          } else {
            w[j][0] = w[j][1] = 0ull;
          }
        }
        // frontier bytes of each word as a bit mask (bit i: byte i == cur)
        u32 msk[SG];
        int c = 0;
#pragma unroll
        for (int j = 0; j < SG; ++j) {
          msk[j] = 0u;
#pragma unroll
          for (int h = 0; h < 16; ++h) {
            const unsigned byte = (unsigned)((w[j][h >> 3] >> (8 * (h & 7))) & 0xffull);
            msk[j] |= (byte == cur ? 1u : 0u) << h;
          }
          c += __popc(msk[j]);
        }
        int total;
        const int off = bscan_excl<BT>(c, &total, s_w);
        for (int p0 = 0; p0 < total; p0 += LCAP) {
          if (off + c > p0 && off < p0 + LCAP) {
            int pos = off;
#pragma unroll
            for (int j = 0; j < SG; ++j) {
              const int base = team_seg(m, G, g0 + j * BT + (int)threadIdx.x);
              for (u32 x = msk[j]; x; x &= x - 1) {
                if (pos >= p0 && pos < p0 + LCAP) s_list[pos - p0] = base + __ffs(x) - 1;
                ++pos;
              }
            }
          }
          __syncthreads();
          const int nl = min(LCAP, total - p0);
          int beg[VPT], dd[VPT];
#pragma unroll
          for (int r = 0; r < VPT; ++r) {
            const int i = r * BT + (int)threadIdx.x;
            const int u = i < nl ? s_list[i] : -1;
            beg[r] = dd[r] = 0;
            if (u >= 0) {
              const int2 x = rp_pair(rp, u);
              beg[r] = x.x;
              dd[r] = x.y - x.x;
            }
          }
          int lmax = 0;
#pragma unroll
          for (int r = 0; r < VPT; ++r)
            if (dd[r] <= LIGHT) lmax = max(lmax, dd[r]);
          lmax = wave_max_nonneg(lmax);
          for (int t0 = 0; t0 < lmax; t0 += 4) {
            int v[4 * VPT];
#pragma unroll
            for (int r = 0; r < VPT; ++r) list4(A.ci, beg[r], dd[r] <= LIGHT ? dd[r] : 0, t0, A.nnz, v + 4 * r);
            team_visit<4 * VPT>(st, rp, lv, v, k, cnt, efn);
          }
          bool heavy = false;
#pragma unroll
          for (int r = 0; r < VPT; ++r) heavy |= dd[r] > LIGHT;
          if (__syncthreads_or(heavy)) {
#pragma unroll
          for (int h = 0; h < VPT / 2; ++h) {
            int run = 0, deg[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
              const int d = dd[2 * h + r];
              run += d > LIGHT ? d : 0;
              deg[r] = run;
            }
            int etot;
            const int eoff = bscan_excl<BT>(run, &etot, s_w);
            if (etot == 0) continue;  // uniform: the workgroup total
#pragma unroll
            for (int r = 0; r < 2; ++r) {
              const int i = threadIdx.x * 2 + r;
              const int inc = eoff + deg[r];
              const int d = deg[r] - (r ? deg[r - 1] : 0);
              s_incl[i] = inc;
              s_off[i] = beg[2 * h + r] - (inc - d);
            }
            __syncthreads();
            for (int e0 = (int)threadIdx.x * U; e0 - (int)threadIdx.x * U < etot; e0 += BT * U) {
              int v[U];
              int o = e0 < etot ? owner_of(s_incl, HCAP, e0) : 0;
#pragma unroll
              for (int j = 0; j < U; ++j) {
                const int e = e0 + j;
                v[j] = -1;
                if (e < etot) {
                  while (s_incl[o] <= e) ++o;
                  v[j] = A.ci[s_off[o] + e];
                }
              }
              team_visit<U>(st, rp, lv, v, k, cnt, efn);
            }
            __syncthreads();
          }
          }
          __syncthreads();
        }
      }
    } else {
      // ---- bottom-up over my vertices: one wave per 64-vertex block, lane =
      // vertex; the first in-edges' stamps read together, the rest scanned
      // wave-cooperatively; a member is the only writer of its vertices here
      const unsigned nxt = stamp_of(k + 1);
      for (int blk = wv; blk < (nseg + 3) / 4; blk += nwv) {
        const int sg = blk * 4 + lane() / 16;
        const int v = sg < nseg ? team_seg(m, G, sg) + (lane() & 15) : n;
        bool open = false;
        if (v < n) open = ld_st(st + v) == 0u;
        bool found = false, pending = false;
        int bb = 0, ee = 0;
        if (open) {
          bb = rp[v];
          ee = rp[v + 1];
          const int d = ee - bb;
          int u[BATCH_T];
#pragma unroll
          for (int t2 = 0; t2 < BATCH_T; ++t2) u[t2] = t2 < d ? A.ci[bb + t2] : -1;
          unsigned su[BATCH_T];
#pragma unroll
          for (int t2 = 0; t2 < BATCH_T; ++t2) su[t2] = u[t2] >= 0 ? ld_st(st + u[t2]) : 0u;
#pragma unroll
          for (int t2 = 0; t2 < BATCH_T; ++t2) found = found || su[t2] == cur;
          pending = !found && d > BATCH_T;
          bb += BATCH_T;
        }
        u64 pm = __ballot(pending);
        while (pm) {
          const int l = __ffsll((long long)pm) - 1;
          pm &= pm - 1;
          const int vb = lane_bcast(bb, l), ve = lane_bcast(ee, l);
          for (int base = vb; base < ve; base += WAVE) {
            const int j = base + lane();
            bool hit = false;
            if (j < ve) hit = ld_st(st + A.ci[j]) == cur;
            if (__ballot(hit)) {
              if (lane() == l) found = true;
              break;
            }
          }
        }
        if (found) {
          put_st(st + v, nxt);
          lv[v] = k + 1;
          ++cnt;
          efn += (u64)(ee - (bb - BATCH_T));
        }
      }
    }
    {
      const u64 wc = wave_sum_u64((u64)cnt), we = wave_sum_u64(efn);
      if (lane() == 0 && wc) {
        atomicAdd(s_cnt, (u32)wc);
        atomicAdd(s_efn, (unsigned long long)we);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      st_dev(&ctl->slot[k & 1][m][0], (u64)*s_cnt);
      st_dev(&ctl->slot[k & 1][m][1], (u64)*s_efn);
    }
    if (!team_barrier<BT>(ctl, G, gen++, s_flag, A.err)) return;
    // every member sums the same counts in the same order
    long long tc = 0, te = 0;
    for (int i = 0; i < G; ++i) {
      tc += (long long)ld_dev(&ctl->slot[k & 1][i][0]);
      te += (long long)ld_dev(&ctl->slot[k & 1][i][1]);
    }
    nF = tc;
    eF = te;
    eU -= eF;
    nU -= nF;
    if (nF == 0) break;
  }
  // the stamps are final: -1 for my vertices never reached, and the out-edges
  // of my reached ones (the component's edges, summed over the members)
  u64 comp = 0;
  for (int i = threadIdx.x; i < nseg * 16; i += BT) {
    const int v = team_seg(m, G, i >> 4) + (i & 15);
    if (v >= n) continue;
    if (ld_st(st + v) == 0u)
      lv[v] = -1;
    else
      comp += (u64)(rp[v + 1] - rp[v]);
  }
  {
    const u64 wc = wave_sum_u64(comp);
    if (lane() == 0 && wc) atomicAdd(A.stats + 2 * b, (unsigned long long)wc);
  }
  if (m == 0 && threadIdx.x == 0) A.stats[2 * b + 1] = (u64)(k + 1);
}

template <int BT>
__global__ __launch_bounds__(BT) void k_batch(BatchArgs A) {
  extern __shared__ __align__(16) char dyn[];
  constexpr int CHMAX = 2 * BT;
  __shared__ int s_buf[2 * CHMAX], s_w[BT / WAVE];  // s_off | s_incl, contiguous (the light rounds' stages)
  int *s_off = s_buf, *s_incl = s_buf + CHMAX;
  __shared__ int s_task[2], s_qn, s_flag;
  __shared__ u32 s_cnt;
  __shared__ unsigned long long s_efn;
  for (;;) {
    if (threadIdx.x == 0) {
      const int t = atomicAdd(A.ticket, 1);
      s_task[0] = t < A.ntask ? A.task[2 * t] : -1;
      s_task[1] = t < A.ntask ? A.task[2 * t + 1] : -1;
    }
    __syncthreads();
    const int b = s_task[0], m = s_task[1];
    __syncthreads();
    if (b < 0) break;
    if (m < 0)
      search_single<BT>(A, b, dyn, s_off, s_incl, s_w, &s_qn, &s_efn);
    else
      search_team<BT>(A, b, m, dyn, s_off, s_incl, s_w, &s_flag, &s_cnt, &s_efn);
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
  if (c.small_vertices < 0 || c.small_vertices > (1 << 20)) return false;
  if (c.team_vertices < 0 || c.max_team < 1 || c.max_team > MAX_TEAM) return false;
  return true;
}

// Defaults: 1024-thread workgroups, and every instance whose visited bitmap
// fits in one workgroup's LDS (up to 2^20 vertices) searched by one workgroup.
static bfs_batch_config default_config() {
  bfs_batch_config c;
  memset(&c, 0, sizeof(c));
  c.block_threads = 1024;
  c.blocks_per_cu = 2;
  c.team_vertices = 131072;
  c.max_team = 8;
  int dev = 0, max_lds = 65536;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  // room for the bitmap beside the kernel's static LDS (about 17 KB at 1024 threads)
  long long room_bits = ((long long)max_lds - 20 * 1024) * 8;
  int small = 1 << 20;
  while (small > 4096 && small > room_bits) small >>= 1;
  c.small_vertices = small;
  return c;
}

static std::mutex g_tune_mu;
static std::map<std::tuple<int, long long, long long>, bfs_batch_config> g_tuned;

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host plan of one launch: task list, team sizes, LDS size and the scratch layout.
struct BatchPlan {
  int grid = 0;
  std::vector<int> head;       // v_off | task pairs | team_g | src | ticket, err
  std::vector<long long> toff; // per-instance state offsets
  size_t head_bytes = 0, toff_at = 0, stats_at = 0, team_at = 0, total = 0;
  size_t lds = 0;              // dynamic LDS bytes per workgroup
  int fr_lds = 0;
  int ntask = 0;
};

template <int BT>
static hipError_t kernel_limits(int *per_cu, size_t lds, size_t *static_lds) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_batch<BT>));
  if (e != hipSuccess) return e;
  *static_lds = fa.sharedSizeBytes;
  if (lds > 65536) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch<BT>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<BT>, BT, lds);
}

static int plan_batch(const bfs_graph_batch *b, const int32_t *sources, const bfs_batch_config &cfg, BatchPlan *P) {
  const int num = b->num;
  std::vector<int> order(num);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int x) {
    return (b->e_off_host[x + 1] - b->e_off_host[x]) + (b->v_off_host[x + 1] - b->v_off_host[x]);
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  const int cus = cus_of_device();
  if (cus <= 0) return hip_fail(hipErrorInvalidDevice, "hipDeviceGetAttribute(multiProcessorCount)");
  int dev = 0, max_lds = 0;
  BFS_HIP(hipGetDevice(&dev));
  BFS_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // LDS: the visited bitmap of the largest single-workgroup instance, and the
  // bottom-up frontier bitmap beside it when both fit
  const size_t vis_bytes = (size_t)((cfg.small_vertices + 63) / 64) * 8;
  int per_cu = 0;
  size_t static_lds = 0;
  hipError_t e = cfg.block_threads == 256 ? kernel_limits<256>(&per_cu, 0, &static_lds)
                 : cfg.block_threads == 512 ? kernel_limits<512>(&per_cu, 0, &static_lds)
                                            : kernel_limits<1024>(&per_cu, 0, &static_lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncGetAttributes(k_batch)");
  const size_t room = (size_t)max_lds > static_lds ? (size_t)max_lds - static_lds : 0;
  if (vis_bytes > room) {
    set_error("bfs_batch: small_vertices %d needs %zu bytes of LDS, %zu available", cfg.small_vertices, vis_bytes,
              room);
    return BFS_EINVAL;
  }
  P->fr_lds = 2 * vis_bytes <= room ? 1 : 0;
  P->lds = P->fr_lds ? 2 * vis_bytes : vis_bytes;
  // team members list their frontier in the same dynamic LDS (4 entries per lane)
  bool any_team = false;
  for (int x = 0; x < num; ++x) any_team |= b->v_off_host[x + 1] - b->v_off_host[x] > cfg.small_vertices;
  if (any_team) P->lds = std::max(P->lds, (size_t)cfg.block_threads * 16);
  if (P->lds > room) {
    set_error("bfs_batch: %zu bytes of LDS needed, %zu available", P->lds, room);
    return BFS_EINVAL;
  }
  e = cfg.block_threads == 256 ? kernel_limits<256>(&per_cu, P->lds, &static_lds)
      : cfg.block_threads == 512 ? kernel_limits<512>(&per_cu, P->lds, &static_lds)
                                 : kernel_limits<1024>(&per_cu, P->lds, &static_lds);
  if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor(k_batch)");
  if (per_cu < 1) {
    set_error("bfs_batch: the kernel cannot be resident with %d threads and %zu bytes of LDS", cfg.block_threads,
              P->lds);
    return BFS_EINVAL;
  }
  // every workgroup of the grid is resident at once (teams wait on each other)
  const int resident = std::min(cfg.blocks_per_cu, per_cu) * cus;
  std::vector<int> team_g(num, 0);
  P->toff.assign(num, 0);
  std::vector<int> tasks;
  size_t state_bytes = 0;
  for (int x : order) {
    const long long n = b->v_off_host[x + 1] - b->v_off_host[x];
    P->toff[x] = (long long)state_bytes;
    if (n <= cfg.small_vertices) {
      state_bytes += single_state_bytes(n, !P->fr_lds);
      tasks.push_back(x);
      tasks.push_back(-1);
      continue;
    }
    long long g = cfg.team_vertices > 0 ? (n + cfg.team_vertices - 1) / cfg.team_vertices : 1;
    g = std::max(1LL, std::min<long long>(g, std::min(cfg.max_team, resident)));
    team_g[x] = (int)g;
    state_bytes += team_state_bytes(n);
    for (int i = 0; i < g; ++i) {
      tasks.push_back(x);
      tasks.push_back(i);
    }
  }
  P->ntask = (int)tasks.size() / 2;
  P->grid = std::min(P->ntask, resident);
  // head ints: v_off[num+1] | task[2 ntask] | team_g[num] | src[num] | ticket | err
  P->head.assign((size_t)(num + 1) + tasks.size() + 2 * (size_t)num + 2, 0);
  int *h = P->head.data();
  for (int i = 0; i <= num; ++i) h[i] = (int)b->v_off_host[i];
  memcpy(h + num + 1, tasks.data(), tasks.size() * 4);
  memcpy(h + num + 1 + tasks.size(), team_g.data(), num * 4);
  memcpy(h + 2 * num + 1 + tasks.size(), sources, num * 4);
  P->head_bytes = P->head.size() * 4;
  P->toff_at = al256(P->head_bytes);
  P->stats_at = P->toff_at + al256((size_t)num * 8);
  P->team_at = P->stats_at + al256((size_t)num * 16);
  P->total = P->team_at + state_bytes;
  return BFS_OK;
}

// Team states (control block and stamps) and the per-instance statistics
// start at zero: a fill kernel (no memset node in a captured stream).
// Block (x, y) clears slice y of instance x's state.
__global__ void k_zero_states(char *team, const long long *toff, const int *team_g, const int *v_off, u64 *stats,
                              int num) {
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < 2 * num; i += blockDim.x) stats[i] = 0ull;
  const int x = blockIdx.x;
  if (x >= num || team_g[x] <= 0) return;
  u64 *p = reinterpret_cast<u64 *>(team + toff[x]);
  const long long words = (long long)team_state_bytes(v_off[x + 1] - v_off[x]) / 8;
  for (long long i = (long long)blockIdx.y * blockDim.x + threadIdx.x; i < words; i += (long long)gridDim.y * blockDim.x)
    p[i] = 0ull;
}

static int batch_run(const bfs_graph_batch *b, const int32_t *sources, int32_t *levels, const bfs_batch_config &cfg,
                     bfs_stats *st, hipStream_t s, float *ms_out) {
  const int num = b->num;
  BatchPlan P;
  int rc = plan_batch(b, sources, cfg, &P);
  if (rc) return rc;
  void *wsp = nullptr;
  if (cfg.workspace) {
    if (cfg.workspace_bytes < P.total) {
      set_error("bfs_batch: workspace has %zu bytes, needs %zu", cfg.workspace_bytes, P.total);
      return BFS_EWORKSPACE;
    }
    wsp = cfg.workspace;
  } else {
    rc = cached_workspace(P.total, &wsp);
    if (rc) return rc;
  }
  char *p = (char *)wsp;
  int *d_head = (int *)p;
  const size_t nt2 = (size_t)P.ntask * 2;
  HostCtx &hc = host_ctx();
  BFS_HIP(hipMemcpyAsync(d_head, P.head.data(), P.head_bytes, hipMemcpyHostToDevice, s));
  BFS_HIP(hipMemcpyAsync(p + P.toff_at, P.toff.data(), (size_t)num * 8, hipMemcpyHostToDevice, s));
  BatchArgs A;
  A.num = num;
  A.ntask = P.ntask;
  A.v_off = d_head;
  A.task = d_head + num + 1;
  A.team_g = d_head + num + 1 + nt2;
  A.src = A.team_g + num;
  A.ticket = const_cast<int *>(A.src) + num;
  A.err = A.ticket + 1;
  A.toff = (const long long *)(p + P.toff_at);
  A.rp = b->row_ptr;
  A.ci = b->col_idx;
  A.levels = levels;
  A.stats = (u64 *)(p + P.stats_at);
  A.team = p + P.team_at;
  A.small_n = cfg.small_vertices;
  A.fr_lds = P.fr_lds;
  A.symmetric = b->symmetric ? 1 : 0;
  A.nnz = b->total_nnz;
  const size_t lds = P.lds;
  BFS_HIP(hipEventRecord(hc.ev[2], s));
  hipLaunchKernelGGL(k_zero_states, dim3(num, 16), dim3(256), 0, s, A.team, A.toff, A.team_g, A.v_off, A.stats, num);
  BFS_HIP(hipGetLastError());
  switch (cfg.block_threads) {
    case 256: hipLaunchKernelGGL(k_batch<256>, dim3(P.grid), dim3(256), lds, s, A); break;
    case 512: hipLaunchKernelGGL(k_batch<512>, dim3(P.grid), dim3(512), lds, s, A); break;
    default: hipLaunchKernelGGL(k_batch<1024>, dim3(P.grid), dim3(1024), lds, s, A); break;
  }
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipEventRecord(hc.ev[3], s));
  std::vector<u64> stats((size_t)num * 2);
  BFS_HIP(hipMemcpyAsync(stats.data(), A.stats, num * 16, hipMemcpyDeviceToHost, s));
  BFS_HIP(hipMemcpyAsync(hc.pinned_u64 + 40, A.err, sizeof(int), hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  if (reinterpret_cast<const int *>(hc.pinned_u64 + 40)[0] != 0) {
    set_error("bfs_batch: a team barrier wait timed out");
    return BFS_EHIP;
  }
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

static int resolve_config(const bfs_graph_batch *b, const bfs_batch_config *cfg_in, bfs_batch_config *cfg) {
  *cfg = default_config();
  if (cfg_in) {
    *cfg = *cfg_in;
  } else {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(b->num, (long long)b->total_n, (long long)b->total_nnz));
    if (it != g_tuned.end()) *cfg = it->second;
  }
  if (!config_ok(*cfg)) {
    set_error("bfs_batch: invalid config (threads %d, blocks/CU %d, small %d, team %d x %d)", cfg->block_threads,
              cfg->blocks_per_cu, cfg->small_vertices, cfg->team_vertices, cfg->max_team);
    return BFS_EINVAL;
  }
  return BFS_OK;
}

}  // namespace bfs

using namespace bfs;

extern "C" int bfs_batch(const bfs_graph_batch *b, const int32_t *sources, int32_t *levels,
                         const bfs_batch_config *cfg_in, bfs_stats *st, void *stream) {
  int rc = check_batch(b, sources, levels);
  if (rc) return rc;
  bfs_batch_config cfg;
  rc = resolve_config(b, cfg_in, &cfg);
  if (rc) return rc;
  return batch_run(b, sources, levels, cfg, st, (hipStream_t)stream, nullptr);
}

extern "C" int bfs_batch_workspace_size(const bfs_graph_batch *b, const int32_t *sources,
                                        const bfs_batch_config *cfg_in, size_t *bytes) {
  if (!bytes) {
    set_error("bfs_batch_workspace_size: bytes is NULL");
    return BFS_EINVAL;
  }
  int rc = check_batch(b, sources, reinterpret_cast<const int32_t *>(b ? b->row_ptr : nullptr));
  if (rc) return rc;
  bfs_batch_config cfg;
  rc = resolve_config(b, cfg_in, &cfg);
  if (rc) return rc;
  BatchPlan P;
  rc = plan_batch(b, sources, cfg, &P);
  if (rc) return rc;
  *bytes = P.total;
  return BFS_OK;
}

extern "C" int bfs_batch_autotune(const bfs_graph_batch *b, const int32_t *sources, int32_t *levels,
                                  bfs_batch_config *best, float *ms_best, void *stream) {
  int rc = check_batch(b, sources, levels);
  if (rc) return rc;
  if (!best) {
    set_error("bfs_batch_autotune: best is NULL");
    return BFS_EINVAL;
  }
  // the caller's workspace (if any) serves every candidate
  void *ws = best->workspace;
  size_t wsb = best->workspace_bytes;
  float best_ms = 1e30f;
  bfs_batch_config bc = default_config();
  bc.workspace = ws;
  bc.workspace_bytes = wsb;
  const int small_max = default_config().small_vertices;
  for (int bt : {512, 1024})
    for (int small : {small_max / 4, small_max})
      for (const int tv : {131072, 65536}) {
          const int mt = tv == 131072 ? 8 : 16;  // team sizes: up to 8 x 131072 or 16 x 65536 vertices
          bfs_batch_config c;
          memset(&c, 0, sizeof(c));
          c.block_threads = bt;
          c.blocks_per_cu = bt == 1024 ? 2 : 4;
          c.small_vertices = small;
          c.team_vertices = tv;
          c.max_team = mt;
          c.workspace = ws;
          c.workspace_bytes = wsb;
          if (!config_ok(c)) continue;
          float ms = 0.f;
          rc = batch_run(b, sources, levels, c, nullptr, (hipStream_t)stream, &ms);  // warm-up
          if (rc == BFS_EWORKSPACE || rc == BFS_EINVAL) continue;  // needs more workspace or LDS than there is
          if (rc) return rc;
          rc = batch_run(b, sources, levels, c, nullptr, (hipStream_t)stream, &ms);
          if (rc) return rc;
          if (ms < best_ms) {
            best_ms = ms;
            bc = c;
          }
        }
  if (best_ms >= 1e30f) {
    set_error("bfs_batch_autotune: no candidate fits the workspace");
    return BFS_EWORKSPACE;
  }
  *best = bc;
  if (ms_best) *ms_best = best_ms;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[std::make_tuple(b->num, (long long)b->total_n, (long long)b->total_nnz)] = bc;
  return BFS_OK;
}
