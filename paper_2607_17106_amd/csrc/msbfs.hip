// Multi-source BFS with up to 64 bit-packed lanes per vertex.
//
// Cascade 1's initialisation admits more than one source node; giving F
// and P one more rank for the source index and packing 64 of its coordinates
// into one u64 per vertex turns a level into word-wide boolean algebra:
//   next[v] = (OR_{u in N_in(v)} front[u]) AND NOT vis[v]     (advance, pull)
//   vis[v]  = vis[v] OR next[v]                                (update)
// and depth k+1 is recorded for every lane bit newly set at v.
//
// Pull (bottom-up, CSC): vertices with more than MS_HEAVY in-edges are split
// into 1024-edge chunks, one wave each (k_ms_pull_heavy); the others go by
// tiles of consecutive vertices cut to similar in-edge counts, a workgroup per
// tile (k_ms_pull_tile): each vertex's thread reads its first MS_HEAD
// in-edges, then the remaining lists of the vertices still missing lanes are
// laid end to end and walked by the whole workgroup.  A vertex stops once
// every lane it lacks is found.  On sparse frontiers an in-neighbour's word is
// gathered only when its bit is set in the any-lane frontier bitmap (n/8
// bytes, cache resident); on dense ones it is gathered directly.
// Push (top-down, CSR): frontier vertices OR their frontier word, masked by
// the target's (read-only) visited word, into the target's next word with
// atomicOr; an owner-computes pass then applies the update.
// Split (bottom-up at a vertex id, see MsArgs::split_t): in-edges from the
// hubs below it are pulled, the out-edges of the frontier vertices above it
// pushed.
//
// Depths are not written during the levels.  Each discovery ORs the new lane
// bits into bit planes of the relative depth r = k + 1 - base (bit l of plane
// b is bit b of lane l's r); one output pass then writes every row of the
// [lanes][n] depth array once, in whole coalesced lines.  When r would need
// more than MS_PLANES planes, a flush pass writes the lanes found so far,
// marks them, and a new window starts at base = k.
#include <string.h>
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "selector.hpp"

namespace bfs {

constexpr int MS_T = 4;   // out-edges per lane before the wave-cooperative walk (push)
constexpr int MS_HEAD = 8; // in-edges a light vertex's own thread reads before the merged walk (pull)
static_assert(MS_HEAD % 4 == 0, "the head is read in 16-byte pieces");
constexpr int MS_PLANES = 8;       // relative depths 0..255 per window
constexpr int MS_HEAVY = 2048;     // in-degree above which a vertex's in-edges are split over waves
constexpr int MS_HCHUNK = 1024;    // in-edges per wave in the heavy pass (<= MS_HEAVY)
constexpr int MS_EPT = 4;          // in-edges per thread per tile iteration (a multiple of 4)
struct __attribute__((packed, aligned(4))) I4u {  // four ints at any 4-byte-aligned address
  int x, y, z, w;
};
constexpr int MS_HB = 1024;        // vertices per workgroup in the heavy-list build
constexpr int MS_SUM_WORDS = 8192; // frontier summary: 2^18 bits = 32 KB of LDS
constexpr int MS_SUM_GRID = 1024;  // persistent workgroups of the summary-filtered bottom-up kernels
// Bottom-up tiles: runs of whole 64-vertex chunks.  A chunk weighs the larger
// of talpha per vertex and the in-degrees of its light (not heavy-listed)
// vertices, and tile t takes the chunks whose running weight starts in
// [t, t + 1) * BLOCK * talpha: BLOCK vertices where in-degrees are low, fewer
// where they are high (a graph ordered by degree puts those together), so no
// tile walks many more in-edges than BLOCK * talpha + 64 * MS_HEAVY.
// (talpha: MsTune::talpha, bfs_multi_config.tile_alpha.)
// Split levels' push (k_ms_push_split): hub targets ORed in LDS (64 KB), workgroups
// of 1024 threads, MS_PQ_GRID of them, staging rows merged MS_PQ_ROWS per thread.
constexpr int MS_PQ_HUB = 8192;   // 64 KB of LDS
constexpr int MS_PQ_BLOCK = 1024;
constexpr int MS_PQ_GRID = 256;
constexpr int MS_PQ_ROWS = 32;    // staging rows merged per k_ms_hub_or thread
constexpr int MS_TALPHA_MIN = 16, MS_TALPHA_MAX = 1024;
// tiles for n vertices and any int32 edge count at any talpha >= MS_TALPHA_MIN
// (a chunk weighs at most 64 * talpha plus its in-edges)
constexpr long long ms_tile_cap(long long n) {
  return n / BLOCK + (1ll << 31) / ((long long)BLOCK * MS_TALPHA_MIN) + 4;
}

// The tunable choices of the level steps (bfs_multi_config, whose zero
// fields take these defaults); none changes the depths.
struct MsTune {
  int wide_ratio = 8;   // non-split bottom-up: wide_vpt vertices per thread while eu > wide_ratio * n
  int split_vpt = 4;    // split levels: vertices per thread (1, 2 or 4)
  int cap0 = 32;        // first-round in-edges per pending vertex on dense-frontier levels
  int talpha = 64;      // tile weight per vertex (see above)
  int alpha = 7;        // bottom-up once frontier out-edges exceed eu / alpha (and n / 8)
  int split_lout = 16;  // split when light frontier out-edges * split_lout < eu
  int wide_vpt = 1;     // vertices per thread on non-split levels with eu > wide_ratio * n
  int narrow_vpt = 4;   // and on the others
};
// Chunk-to-owner tables of the heavy lists: entries for chunks below this
// many; later chunks (graphs with far more edges than vertices) search hpre.
constexpr long long ms_hq_cap(long long n) { return n * 2 + 1024 < (1ll << 22) ? n * 2 + 1024 : (1ll << 22); }
static_assert(MS_HCHUNK <= MS_HEAVY, "a heavy list is longer than one chunk");

struct MsCtr {  // two 64-byte lines per shard
  u64 newbits;     // (lane, vertex) pairs discovered
  u64 comp_edges;  // sum over discoveries of outdeg(v) (per lane)
  u64 active;      // vertices with at least one new lane (next frontier size)
  u64 active_out;  // their out-edges
  u64 done_in;     // in-edges of vertices whose last lane was found
  u64 scanned;     // edges examined
  u64 unvis;       // vertices still missing some lane when the step started
  u64 hits;        // examined edges whose source is in the frontier (words gathered)
  u64 hscanned;    // the part of `scanned` examined by the heavy-vertex kernel
  u64 hhits;       // the part of `hits` gathered by it
  u64 hpend;       // bottom-up: heavy vertices still missing some lane after the step
  u64 lout;        // out-edges of the found vertices at or above the split id (hub_t)
  u64 pscan;       // split level: edges examined by the light-source push (part of `scanned`)
  u64 pact;        // split level: frontier vertices that push expanded
  u64 pad[1];
  u64 seq;         // totals only: sequence number written last (host polling)
};
static_assert(sizeof(MsCtr) == 128, "MsCtr is two lines");
constexpr int MS_NCTR = 16;

struct MsArgs {
  int n, k, L;          // vertices, level, lanes in this group
  int rel;              // relative depth of this step's discoveries (k + 1 - base)
  u64 full;             // mask of the L lanes
  const int *rp, *ci, *cp, *cx;
  int ncx;              // entries of cx (the in-edge count)
  int sym;              // cp == rp (a symmetric graph passes one array twice)
  const u64 *front;     // F_k words
  const u64 *fbits;     // any-lane bitmap of F_k: bit v%64 of word v/64
  u64 *next;            // F_{k+1} words
  u64 *nbits;           // any-lane bitmap of F_{k+1}, every word written by the step
  u64 *dead;            // buffer to clear for F_{k+2}
  u64 *vis;
  u64 *planes;          // plane b at planes + b * n
  u64 *flushed;         // lanes whose depths a flush pass has written
  u64 *accb;            // heavy vertices: lanes found by the heavy pass this level (else 0)
  const int *hv;        // heavy vertices in increasing order
  const int *hpre;      // hpre[i]: first chunk of hv[i]; hpre[hcount] = hchunks
  int hcount, hchunks;
  const int *hq, *oq;   // chunk q's index in hv (ov) for q < hqcap
  int hqcap;
  const int *ov;        // the same for out-degree (CSR): heavy sources of the top-down step
  const int *opre;
  int ocount, ochunks;  // -1: not read back yet; k_ms_push_heavy takes them from otot
  const int *otot;      // device {ocount, ochunks}
  int *levels;          // row l at levels + l * n
  const int *vmap;      // or null: column v of `levels` is vertex vmap[v] of the (renumbered) graph
  u32 *hsrc;            // top-down: set by k_ms_push when the frontier holds a heavy source, cleared by
                        // k_ms_push_update; k_ms_push_heavy does nothing while it is 0
  // Split bottom-up level at split_t: in-edges from vertices below split_t
  // are pulled (an in-edge list is read only up to its first entry >=
  // split_t: lists are ascending), and the frontier vertices at or above
  // split_t push their out-edges into `next` first (push_lo =
  // split_t, k_ms_push_split and k_ms_hub_or).  The two
  // halves cover every edge, so any split id gives the same result; on a graph
  // numbered by decreasing degree, the heavy out-degree count turns a sparse
  // hub frontier's full in-edge scan into the hubs' in-edges plus a few light
  // out-edges.
  int hub_t;            // split id of this call (0: none); discoveries at or above it count their
                        // out-edges in lout (-1 before the host has read it: k_ms_push_update
                        // takes otot[0], the heavy out-degree count)
  int split_t;          // this level's split id (0: not a split level)
  int push_lo;          // k_ms_push: first vertex to expand (split level: split_t; else 0)
  u64 *hubst;           // split level: staging rows of k_ms_push_split (MS_PQ_GRID x MS_PQ_HUB words)
  int base, np, nflush; // output passes: window base, planes in use, flushes so far
  int cap0;             // bottom-up: in-edges per pending vertex in the first merged round
  u64 *zplane;          // plane for the step kernels to zero for the next level, or null
  const int *tstart;    // bottom-up tile t covers vertices [tstart[t], tstart[t + 1])
  int ntiles;
  const u32 *fsum;      // summary of fbits: bit i set if any vertex in [i << sshift, (i+1) << sshift) is
  int sshift;           // in the frontier; MS_SUM_WORDS words, staged in LDS by bottom-up kernels
                        // when the frontier is sparse
  MsCtr *sh;            // NSH shards of this level's counters
  // Sparse top-down level: k_ms_push clears the dead buffer at the vertices
  // of its bitmap (nbits before it is rewritten: the dead buffer is nonzero
  // only there) and appends every vertex whose next word it turns nonzero to
  // tq; k_ms_push_update_sparse then updates only those.
  int sparse;
  int *tq;              // touched list (n entries)
  u32 *tqn;             // its length
};

struct MsCarve {
  u64 *fr[3], *vis, *flushed, *accb, *planes, *fb[2];
  u32 *fsum;
  int *hv, *hpre, *ov, *opre, *bcnt, *bchk, *tstart, *hq, *oq;
  u64 *hubst;
  long long *bwt;       // per heavy-list block: tile weight of its chunks, then their exclusive prefix
  MsCtr *sh, *tot;
  int *tq;              // sparse top-down levels: vertices whose next word turned nonzero
  int *src;             // [64] sources of the group, [64] their degrees, [192..196] heavy and tile
                        // totals, [200] the top-down heavy-source flag, [203] the touched-list
                        // length
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
  c.accb = reinterpret_cast<u64 *>(p + off);
  off += vb;
  const size_t ib = al(((size_t)n + 1) * 4), nb = al(((size_t)n / MS_HB + 2) * 4);
  c.hv = reinterpret_cast<int *>(p + off);
  off += ib;
  c.hpre = reinterpret_cast<int *>(p + off);
  off += ib;
  c.ov = reinterpret_cast<int *>(p + off);
  off += ib;
  c.opre = reinterpret_cast<int *>(p + off);
  off += ib;
  c.hubst = reinterpret_cast<u64 *>(p + off);
  off += (size_t)MS_PQ_GRID * MS_PQ_HUB * 8;
  c.bcnt = reinterpret_cast<int *>(p + off);
  off += nb;
  c.bchk = reinterpret_cast<int *>(p + off);
  off += nb;
  c.hq = reinterpret_cast<int *>(p + off);
  off += al((size_t)ms_hq_cap(n) * 4);
  c.oq = reinterpret_cast<int *>(p + off);
  off += al((size_t)ms_hq_cap(n) * 4);
  c.tstart = reinterpret_cast<int *>(p + off);
  off += al((size_t)ms_tile_cap(n) * 4);
  c.bwt = reinterpret_cast<long long *>(p + off);
  off += al(((size_t)n / MS_HB + 2) * 8);
  c.planes = reinterpret_cast<u64 *>(p + off);
  off += al((size_t)MS_PLANES * n * 8);
  for (int i = 0; i < 2; ++i, off += bb) c.fb[i] = reinterpret_cast<u64 *>(p + off);
  c.fsum = reinterpret_cast<u32 *>(p + off);
  off += al((size_t)MS_SUM_WORDS * 4);
  c.sh = reinterpret_cast<MsCtr *>(p + off);
  c.tot = c.sh + NSH;
  off += (size_t)(NSH + 1) * sizeof(MsCtr);
  c.tq = reinterpret_cast<int *>(p + off);
  off += ib;
  c.src = reinterpret_cast<int *>(p + off);
  off += 1024;
  c.bytes = off;
  return c;
}

size_t workspace_bytes_multi(int n) { return ms_carve(0, n).bytes; }

__device__ __forceinline__ bool in_front(const u64 *fb, int u) { return (fb[u >> 6] >> (u & 63)) & 1ull; }

// Frontier test with the LDS summary first (SUM) or the bitmap alone.
template <bool SUM>
__device__ __forceinline__ bool in_front_s(const MsArgs &a, const u32 *s_sum, int u) {
  if (SUM && !((s_sum[u >> (a.sshift + 5)] >> ((u >> a.sshift) & 31)) & 1u)) return false;
  return in_front(a.fbits, u);
}

// Frontier test of in-neighbour u (-1: none) before its word is gathered: the
// summary and bitmap (PROBE), or none on dense frontiers, where nearly every
// examined in-neighbour is in the frontier and its word, zero off the frontier,
// is the test itself.
template <bool SUM, bool PROBE>
__device__ __forceinline__ bool ms_probe(const MsArgs &a, const u32 *s_sum, int u) {
  return u >= 0 && (!PROBE || in_front_s<SUM>(a, s_sum, u));
}

template <bool SUM>
__device__ __forceinline__ void ms_stage_summary(const MsArgs &a, u32 *s_sum) {
  if (SUM) {
    for (int i = threadIdx.x; i < MS_SUM_WORDS; i += BLOCK) s_sum[i] = a.fsum[i];
    __syncthreads();
  }
}

// Summary of the frontier bitmap (one thread per summary word): bit i of the
// summary is the OR of bitmap bits [i << sshift, (i+1) << sshift), sshift >= 4.
__global__ __launch_bounds__(BLOCK) void k_ms_summary(const u64 *fb, int nwords, u32 *sum, int sshift) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= MS_SUM_WORDS) return;
  u32 out = 0;
  if (sshift < 6) {  // 64 >> sshift groups per bitmap word
    const int gpw = 64 >> sshift, wpw = 32 / gpw;  // groups per word, bitmap words per summary word
    for (int k = 0; k < wpw; ++k) {
      const long long w = (long long)i * wpw + k;
      const u64 x = w < nwords ? fb[w] : 0ull;
      for (int gi = 0; gi < gpw; ++gi)
        if ((x >> (gi << sshift)) & ((1ull << (1 << sshift)) - 1ull)) out |= 1u << (k * gpw + gi);
    }
  } else {  // each group spans 1 << (sshift - 6) bitmap words
    const int wpg = 1 << (sshift - 6);
    for (int gi = 0; gi < 32; ++gi) {
      const long long w0 = ((long long)i * 32 + gi) * wpg;
      u64 x = 0ull;
      for (int k = 0; k < wpg && w0 + k < nwords; ++k) x |= fb[w0 + k];
      if (x) out |= 1u << gi;
    }
  }
  sum[i] = out;
}

enum { C_NEW, C_COMP, C_ACTIVE, C_ACTOUT, C_DONEIN, C_SCAN, C_UNVIS, C_HITS, C_HSCAN, C_HHITS, C_HPEND, C_LOUT,
       C_PSCAN, C_PACT };

// Per-thread counters.  Within one launch every vertex is found, and every
// edge examined, at most once, so each count but C_COMP stays below the edge
// count (< 2^31) per thread and is kept in 32 bits (registers: the tile kernel
// keeps ten of them live); C_COMP (lanes x out-degree) is kept in 64.
struct MsStats {
  u32 c[MS_NCTR] = {};
  u64 comp = 0;
  __device__ __forceinline__ u64 get(int j) const { return j == C_COMP ? comp : (u64)c[j]; }
};

// Counters a kernel may touch, as a bit mask of their indices: the flush
// reduces only those (a 64-lane reduction of a u64 costs some 24 VALU
// instructions per counter and wave).
constexpr unsigned ms_bit(int c) { return 1u << c; }
constexpr unsigned MS_M_FOUND =
    ms_bit(C_NEW) | ms_bit(C_COMP) | ms_bit(C_ACTIVE) | ms_bit(C_ACTOUT) | ms_bit(C_DONEIN) | ms_bit(C_LOUT);
constexpr unsigned MS_M_ALL = (1u << MS_NCTR) - 1;

// Workgroup-level flush: one atomic per counter and workgroup.  Every thread
// of the workgroup must call it.
template <unsigned MASK = MS_M_ALL>
__device__ __forceinline__ void ms_flush_block(MsStats &st, MsCtr *sh) {
  __shared__ u64 s_red[BLOCK / WAVE][MS_NCTR];
#pragma unroll
  for (int j = 0; j < MS_NCTR; ++j) {
    if (!((MASK >> j) & 1u)) continue;
    const u64 r = wave_sum_u64(st.get(j));
    if (lane() == 0) s_red[threadIdx.x / WAVE][j] = r;
  }
  __syncthreads();
  if (threadIdx.x < MS_NCTR && ((MASK >> threadIdx.x) & 1u)) {
    u64 r = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / WAVE; ++w) r += s_red[w][threadIdx.x];
    if (r) atomicAdd(reinterpret_cast<u64 *>(sh + (blockIdx.x % NSH)) + threadIdx.x, r);
  }
}

// Reduces the NSH counter shards of a level into *tot (pinned host memory)
// and clears each shard after reading it, ready for the next level.  One
// thread writes the totals, then -- after a system-scope fence -- `seq` into
// the last word, which the host polls instead of waiting for the stream.
// tqn (after a sparse top-down level): the touched-list length, reset.
__global__ __launch_bounds__(NSH) void k_ms_finish(MsCtr *sh, MsCtr *tot, u64 seq, u32 *tqn) {
  __shared__ u64 s_red[MS_NCTR][NSH / WAVE];
  const int t = threadIdx.x;
  u64 *f = reinterpret_cast<u64 *>(sh + t);
  u64 x[MS_NCTR];  // all of the shard's loads in flight before the first reduction
#pragma unroll
  for (int j = 0; j < MS_NCTR; ++j) x[j] = f[j];
#pragma unroll
  for (int j = 0; j < MS_NCTR; ++j) f[j] = 0ull;
#pragma unroll
  for (int j = 0; j < MS_NCTR; ++j) {
    const u64 r = wave_sum_u64(x[j]);
    if (lane() == 0) s_red[j][t / WAVE] = r;
  }
  __syncthreads();
  if (t == 0) {
    if (tqn) *tqn = 0u;
    u64 *o = reinterpret_cast<u64 *>(tot);
    for (int j = 0; j < MS_NCTR - 1; ++j) {
      u64 r = 0;
      for (int i = 0; i < NSH / WAVE; ++i) r += s_red[j][i];
      o[j] = r;
    }
    __threadfence_system();
    reinterpret_cast<volatile u64 *>(o)[MS_NCTR - 1] = seq;
  }
}

// Clears the dead frontier buffer and, when the host asks for it, the depth
// plane the next level will use for the first time (zeroed here, one level
// ahead, instead of by a launch on the host's critical path).  dead = null:
// another kernel of the level does it.
__device__ __forceinline__ void ms_clear_dead(const MsArgs &a) {
  if (!a.dead) return;
  const int tid = blockIdx.x * BLOCK + threadIdx.x;  // BLOCK-wide workgroups
  const int nthr = gridDim.x * BLOCK;
  for (int i = tid; i < a.n; i += nthr) {
    a.dead[i] = 0ull;
    if (a.zplane) a.zplane[i] = 0ull;
  }
}

// Records the discovery of `nw` lanes at v (owner thread, so the plane
// updates are plain read-modify-writes): vis, depth planes, stats.
// in_deg >= 0: v's in-degree, already at hand (the bottom-up tile loaded its
// in-edge offsets), which is also its out-degree on a symmetric graph; -1:
// both are read here.
__device__ __forceinline__ void ms_discover(const MsArgs &a, int v, u64 vis_old, u64 nw, MsStats &st,
                                            int in_deg = -1) {
  const u64 vnew = vis_old | nw;
  a.vis[v] = vnew;
  for (int r = a.rel, b = 0; r; r >>= 1, ++b)
    if (r & 1) a.planes[(size_t)b * a.n + v] |= nw;
  const int c = __popcll(nw);
  const int od = (in_deg >= 0 && a.sym) ? in_deg : a.rp[v + 1] - a.rp[v];
  st.c[C_NEW] += (u32)c;
  st.comp += (u64)c * (u64)od;
  st.c[C_ACTIVE] += 1;
  st.c[C_ACTOUT] += (u32)od;
  if (v >= a.hub_t) st.c[C_LOUT] += (u32)od;
  if ((vnew & a.full) == a.full) st.c[C_DONEIN] += (u32)(in_deg >= 0 ? in_deg : a.cp[v + 1] - a.cp[v]);
}

// Writes the depth of every lane of v not in `skip`: a.base + r for visited
// lanes (r read from the NP planes in use), -1 for the others.  Called by
// whole waves holding 64 consecutive vertices, so each of the L row stores
// covers 64 consecutive ints; lanes with valid = false store nothing.  The
// planes are split into 32-bit halves so one bit-field extract per plane
// gives a lane's bit.
template <int NP>
__device__ __forceinline__ void ms_store_depths(const MsArgs &a, int v, int m, bool valid, u64 vw, u64 skip) {
  uint32_t pl[2][NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const u64 w = (valid && vw) ? a.planes[(size_t)b * a.n + m] : 0ull;
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
      if ((st_h >> l) & 1u) __builtin_nontemporal_store(((vis_h >> l) & 1u) ? a.base + r : -1, out);
    }
  }
}

template <int NP>
__device__ __forceinline__ void ms_out_body(const MsArgs &a, int flush) {
  for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {  // uniform per wave
    const int v = base + threadIdx.x;  // output column; flushed is indexed by it too
    const bool valid = v < a.n;
    const int m = valid && a.vmap ? a.vmap[v] : v;
    const u64 vw = valid ? a.vis[m] & a.full : 0ull;
    const u64 fl = (valid && a.nflush) ? a.flushed[v] : 0ull;
    if (flush) {
      ms_store_depths<NP>(a, v, m, valid, vw, ~(vw & ~fl));
      if (valid) a.flushed[v] = vw;
    } else {
      ms_store_depths<NP>(a, v, m, valid, vw, fl);
    }
  }
}

// ------------------------------------------------------------------ init
// Clears a group's state: visited words, the three frontier buffers, both
// frontier bitmaps, depth planes 0 and 1 (relative depths 1..3), the
// counter shards (k_ms_finish keeps those clear afterwards), the
// heavy-source flag and the touched-list length.  With every frontier buffer
// and bitmap zero, the first level, like any later sparse top-down level,
// clears only what it finds set.
__global__ __launch_bounds__(BLOCK) void k_ms_init(MsArgs a, u64 *f0, u64 *f1, u64 *f2, u64 *b0, u64 *b1) {
  const int nw = (a.n + 63) / 64;
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
    a.vis[v] = 0ull;
    f0[v] = 0ull;
    f1[v] = 0ull;
    f2[v] = 0ull;
    a.planes[v] = 0ull;
    a.planes[(size_t)a.n + v] = 0ull;
    if (v < nw) {
      b0[v] = 0ull;
      b1[v] = 0ull;
    }
  }
  u64 *sh = reinterpret_cast<u64 *>(a.sh);
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < NSH * MS_NCTR; i += gridDim.x * BLOCK) sh[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.hsrc = 0u;
    *a.tqn = 0u;
  }
}

// One thread per lane: sets the source bit (duplicates OR); depth 0 is
// relative depth 0, which the zeroed planes already hold.
struct MsSources {
  int v[64];
};

// One thread per lane: maps the lane's source to the graph's numbering (a
// renumbered graph), sets its bit (duplicates OR; depth 0 is relative depth 0,
// which the zeroed planes already hold), and posts to host memory what the
// host needs before the first level: the sources' out-degrees (post[64 + l])
// and, copied from `tot`, the heavy-list and tile totals (post[0 .. 4]); then,
// after system-scope fences, the sequence word.
__global__ void k_ms_seed(MsArgs a, MsSources src, u64 *f0, u64 *b0, const int *tot, int *post,
                          u64 *post_seq, u64 seq) {
  const int l = threadIdx.x;
  if (l < a.L) {
    int s = src.v[l];
    if (a.vmap) s = a.vmap[s];
    atomicOr(a.vis + s, 1ull << l);
    atomicOr(f0 + s, 1ull << l);
    atomicOr(b0 + (s >> 6), 1ull << (s & 63));
    post[64 + l] = a.rp[s + 1] - a.rp[s];
  }
  if (l < 5) post[l] = tot[l];
  __threadfence_system();  // each lane's posts reach the host before the sequence word
  __syncthreads();
  if (l == 0) *reinterpret_cast<volatile u64 *>(post_seq) = seq;
}

__global__ __launch_bounds__(BLOCK) void k_ms_fill(u64 *p, int n) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) p[i] = 0ull;
}

// First position in [lo, hi) of an ascending int array holding a value >= t
// (hi if none): one thread.
__device__ __forceinline__ int ms_lower_bound(const int *x, int lo, int hi, int t) {
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (x[mid] < t) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// The same for a whole wave (same arguments in every lane, same result): each
// round the lanes test 64 evenly spaced entries at once and a ballot narrows
// the range 64-fold, so 4096 entries take two rounds of one load each.
__device__ __forceinline__ int ms_wave_lower_bound(const int *x, int lo, int hi, int t) {
  while (lo < hi) {  // the answer lies in [lo, hi]
    const int step = (hi - lo + WAVE - 1) / WAVE;
    const int p = lo + lane() * step;
    const u64 below = __ballot(p < hi && x[p] < t);  // a prefix of the lanes (x ascending)
    const int k = __popcll(below);
    if (k == 0) return lo;
    const int pk = lo + k * step;  // first tested position not below t, if any
    lo = lo + (k - 1) * step + 1;
    hi = min(hi, pk);
  }
  return lo;
}

// ------------------------------------------------------------ heavy list
// Vertices with in-degree (CSC) or out-degree (CSR) > MS_HEAVY, in increasing
// order, and the prefix of their chunk counts: a count pass per MS_HB vertices, a one-workgroup scan of
// the per-workgroup totals, and a write pass.  Built once per call.
// Each thread takes 4 consecutive vertices of its workgroup's MS_HB (one pass,
// one scan per array); 16 neighbouring lanes hold one 64-vertex tile chunk.
static_assert(MS_HB == 4 * BLOCK, "four vertices per thread in the heavy-list build");

// Vertices v .. v+3 (those below v1 <= n): h[i] = chunks of v+i if heavy
// (else 0); *light = the sum of the light ones' degrees.
__device__ __forceinline__ void ms_quad(const int *cp, int v, int v1, int (&h)[4], u64 *light) {
  int c[5];
  if (v + 4 <= v1) {  // all four: one 16-byte load (4-byte aligned) and one more
    const I4u q = *reinterpret_cast<const I4u *>(cp + v);
    c[0] = q.x;
    c[1] = q.y;
    c[2] = q.z;
    c[3] = q.w;
    c[4] = cp[v + 4];
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) c[i] = v + i <= v1 ? cp[v + i] : 0;
  }
  u64 l = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int d = v + i < v1 ? c[i + 1] - c[i] : 0;
    h[i] = d > MS_HEAVY ? (d + MS_HCHUNK - 1) / MS_HCHUNK : 0;
    l += d <= MS_HEAVY ? (u64)d : 0ull;
  }
  *light = l;
}

// Tile weight of the 64-vertex chunk starting at cw (see MS_TALPHA) from the
// 16 lanes holding it: every lane of the group passes its `light`; the
// result is valid in all 16.
__device__ __forceinline__ long long ms_chunk_weight16(u64 light, int cw, int n, int talpha) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) light += __shfl_xor(light, o);
  const long long floor_w = (long long)min(n - cw, WAVE) * talpha;
  return max(floor_w, (long long)light);
}

__device__ __forceinline__ long long block_excl_scan_ll(long long x, long long *total, long long *s_w) {
  const int w = threadIdx.x / WAVE;
  const long long incl = (long long)wave_incl_scan_u64((u64)x);
  if (lane() == WAVE - 1) s_w[w] = incl;
  __syncthreads();
  long long off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / WAVE; ++i) {
    off += (i < w) ? s_w[i] : 0;
    tot += s_w[i];
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

// Per MS_HB vertices: heavy vertices, their chunks and (bwt given) the tile
// weight of the 64-vertex chunks.
__global__ __launch_bounds__(BLOCK) void k_ms_heavy_count(const int *cp, int n, int *bcnt, int *bchk,
                                                          long long *bwt, int talpha) {
  __shared__ int s_w[BLOCK / WAVE];
  __shared__ long long s_wl[BLOCK / WAVE];
  const int v0 = blockIdx.x * MS_HB, v1 = min(v0 + MS_HB, n);
  const int v = v0 + 4 * (int)threadIdx.x;
  int h[4] = {0, 0, 0, 0};
  u64 light = 0;
  if (v < v1) ms_quad(cp, v, v1, h, &light);
  int c = 0, k = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    c += h[i] ? 1 : 0;
    k += h[i];
  }
  long long wt = 0;
  if (bwt) {  // uniform
    const int cw = v0 + WAVE * (int)(threadIdx.x / 16);
    const long long w = ms_chunk_weight16(light, cw, n, talpha);
    if ((threadIdx.x & 15) == 0 && cw < v1) wt = w;
  }
  int tc, tk;
  long long tw;
  block_excl_scan(c, &tc, s_w);
  block_excl_scan(k, &tk, s_w);
  block_excl_scan_ll(wt, &tw, s_wl);
  if (threadIdx.x == 0) {
    bcnt[blockIdx.x] = tc;
    bchk[blockIdx.x] = tk;
    if (bwt) bwt[blockIdx.x] = tw;
  }
}

// In place: bcnt/bchk (and bwt) become exclusive offsets; tot = {heavy
// vertices, chunks}, *tiles = bottom-up tiles (total weight / (BLOCK * talpha) + 1).
// One workgroup, MS_SCAN_CH entries at a time staged in LDS (coalesced loads
// and stores): each thread sums a contiguous segment, one block scan per array
// gives the segments' offsets, each thread rewrites its segment.
constexpr int MS_SCAN_CH = 4096;
__global__ __launch_bounds__(BLOCK) void k_ms_heavy_scan(int nb, int *bcnt, int *bchk, int *tot, long long *bwt,
                                                         int *tiles, int talpha) {
  __shared__ int s_c[MS_SCAN_CH], s_k[MS_SCAN_CH];
  __shared__ long long s_x[MS_SCAN_CH];
  __shared__ int s_w[BLOCK / WAVE];
  __shared__ long long s_wl[BLOCK / WAVE];
  constexpr int SEG = MS_SCAN_CH / BLOCK;
  int rc = 0, rk = 0;
  long long rw = 0;
  for (int base = 0; base < nb; base += MS_SCAN_CH) {  // uniform
    const int m = min(MS_SCAN_CH, nb - base);
    {  // all loads in flight before the first LDS store: registers first, from
       // in-range addresses (clamped, so no branch around a load)
      int xc[SEG], xk[SEG];
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const int i = base + min((int)threadIdx.x + j * BLOCK, m - 1);
        xc[j] = bcnt[i];
        xk[j] = bchk[i];
      }
      if (bwt) {  // uniform
        long long xw[SEG];
#pragma unroll
        for (int j = 0; j < SEG; ++j) xw[j] = bwt[base + min((int)threadIdx.x + j * BLOCK, m - 1)];
#pragma unroll
        for (int j = 0; j < SEG; ++j)
          if ((int)threadIdx.x + j * BLOCK < m) s_x[threadIdx.x + j * BLOCK] = xw[j];
      }
#pragma unroll
      for (int j = 0; j < SEG; ++j)
        if ((int)threadIdx.x + j * BLOCK < m) {
          s_c[threadIdx.x + j * BLOCK] = xc[j];
          s_k[threadIdx.x + j * BLOCK] = xk[j];
        }
    }
    __syncthreads();
    const int i0 = threadIdx.x * SEG, i1 = min(m, i0 + SEG);
    int c = 0, k = 0;
    long long w = 0;
    for (int i = i0; i < i1; ++i) {
      c += s_c[i];
      k += s_k[i];
      if (bwt) w += s_x[i];
    }
    int tc, tk;
    long long tw = 0;
    int oc = rc + block_excl_scan(c, &tc, s_w);
    int ok = rk + block_excl_scan(k, &tk, s_w);
    long long ow = bwt ? rw + block_excl_scan_ll(w, &tw, s_wl) : 0;  // bwt is the same in every thread
    for (int i = i0; i < i1; ++i) {
      const int xc = s_c[i], xk = s_k[i];
      s_c[i] = oc;
      s_k[i] = ok;
      oc += xc;
      ok += xk;
      if (bwt) {
        const long long xw = s_x[i];
        s_x[i] = ow;
        ow += xw;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += BLOCK) {
      bcnt[base + i] = s_c[i];
      bchk[base + i] = s_k[i];
      if (bwt) bwt[base + i] = s_x[i];
    }
    rc += tc;
    rk += tk;
    rw += tw;
    __syncthreads();  // the next chunk reuses the LDS arrays
  }
  if (threadIdx.x == 0) {
    tot[0] = rc;
    tot[1] = rk;
    if (bwt) *tiles = (int)(rw / ((long long)BLOCK * talpha)) + 1;
  }
}
static_assert(MS_SCAN_CH % BLOCK == 0, "whole segments");

// Also clears accb of every heavy vertex (the only entries the pull uses)
// when accb is given.
// With bwt: chunk c starting at running weight key writes tstart[t] = its end
// for each tile t whose first weight t * BLOCK * talpha lies in (key, key + w_c]
// (tiles inside one chunk's span are empty); tstart[0] = 0, tstart[tiles] = n.
__global__ __launch_bounds__(BLOCK) void k_ms_heavy_write(const int *cp, int n, const int *bcnt, const int *bchk,
                                                          int *hv, int *hpre, int *hq, int hqcap, u64 *accb,
                                                          const int *tot, const long long *bwt, int *tstart,
                                                          const int *tiles, int talpha) {
  __shared__ int s_w[BLOCK / WAVE];
  __shared__ long long s_wl[BLOCK / WAVE];
  const int v0 = blockIdx.x * MS_HB, v1 = min(v0 + MS_HB, n);
  const int v = v0 + 4 * (int)threadIdx.x;
  int h[4] = {0, 0, 0, 0};
  u64 light = 0;
  if (v < v1) ms_quad(cp, v, v1, h, &light);
  int c = 0, k = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    c += h[i] ? 1 : 0;
    k += h[i];
  }
  int tc, tk;
  int pos = bcnt[blockIdx.x] + block_excl_scan(c, &tc, s_w);
  int chk = bchk[blockIdx.x] + block_excl_scan(k, &tk, s_w);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (h[i]) {
      hv[pos] = v + i;
      hpre[pos] = chk;
      for (int q = chk; q < chk + h[i] && q < hqcap; ++q) hq[q] = pos;
      if (accb) accb[v + i] = 0ull;
      ++pos;
      chk += h[i];
    }
  if (bwt) {  // uniform
    const int cw = v0 + WAVE * (int)(threadIdx.x / 16);
    const long long w = ms_chunk_weight16(light, cw, n, talpha);
    const bool lead = (threadIdx.x & 15) == 0 && cw < v1;
    const long long tw_all = (long long)BLOCK * talpha;
    long long tw;
    const long long key = bwt[blockIdx.x] + block_excl_scan_ll(lead ? w : 0, &tw, s_wl);
    if (lead) {
      const int e = min(cw + WAVE, n), last = *tiles - 1;
      for (long long t = key / tw_all + 1; t <= (key + w) / tw_all && t <= last; ++t) tstart[t] = e;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hpre[tot[0]] = tot[1];
    if (bwt) {
      tstart[0] = 0;
      tstart[*tiles] = n;
    }
  }
}

// ------------------------------------------------------------------ pull
// Index i of the heavy vertex owning chunk q: the last i with hpre[i] <= q
// (hpre[hcount] = hchunks > q).  Wave-uniform 64-ary search: each round the
// 64 lanes test 64 evenly spaced entries of the current interval and a ballot
// narrows it 64-fold, so 12K heavy vertices take 3 rounds of one load each.
__device__ __forceinline__ int ms_heavy_of_chunk(const int *hpre, int hcount, int q);

// The same from the chunk-to-owner table where it has the entry.
__device__ __forceinline__ int ms_chunk_owner(const int *hq, int hqcap, const int *hpre, int hcount, int q) {
  return q < hqcap ? hq[q] : ms_heavy_of_chunk(hpre, hcount, q);
}

__device__ __forceinline__ int ms_heavy_of_chunk(const int *hpre, int hcount, int q) {
  int lo = 0, hi = hcount;  // hpre[lo] <= q < hpre[hi]
  while (hi - lo > 1) {
    const int step = (hi - lo + WAVE - 1) / WAVE;
    const int idx = lo + lane() * step;
    const bool le = idx < hi && hpre[idx] <= q;
    const u64 m = __ballot(le);  // lanes 0..k are set (hpre is non-decreasing); lane 0 always
    const int k = 63 - __clzll((long long)m);
    lo = lo + k * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// Bottom-up, heavy part: one wave per chunk of MS_HCHUNK in-edges of a heavy
// vertex that still misses lanes.  The wave ORs the frontier words of 64
// in-edges at a time, MS_HU rounds per iteration with their loads in flight
// together (bitmap probe first).  Every MS_POST iterations it posts its
// lanes to accb[v] with a returning atomic OR, which also tells it what the
// other chunks of v have found; it stops once v's missing lanes are covered.
constexpr int MS_HU = 4;    // 64-edge rounds per heavy-pass iteration
constexpr int MS_POST = 1;  // iterations between posts

// phase 0: every chunk; 1: the first chunk of each heavy vertex; 2: the other
// chunks.  On dense frontiers a vertex's first chunk usually finds every lane
// it misses, so running the first chunks on their own lets the others see that
// in accb before reading any edge (all chunks at once each read a round).
template <bool SUM, bool PROBE = true>
__global__ __launch_bounds__(BLOCK) void k_ms_pull_heavy(MsArgs a, int phase) {
  extern __shared__ u32 s_sum[];
  ms_stage_summary<SUM>(a, s_sum);
  MsStats st;
  const int wv = threadIdx.x / WAVE;
  const int items = phase == 1 ? a.hcount : a.hchunks;
  for (int it = blockIdx.x * (BLOCK / WAVE) + wv; it < items; it += gridDim.x * (BLOCK / WAVE)) {
    int i, q;
    if (phase == 1) {
      i = it;
      q = a.hpre[i];
    } else {
      q = it;
      i = ms_chunk_owner(a.hq, a.hqcap, a.hpre, a.hcount, q);
    }
    const int q0 = a.hpre[i];  // the vertex's first chunk
    if (phase == 2 && q == q0) continue;
    const int v = a.hv[i];
    const u64 need = a.full & ~a.vis[v];
    if (!need) continue;
    const int sb = a.cp[v] + (q - q0) * MS_HCHUNK;
    int se = min(a.cp[v + 1], sb + MS_HCHUNK);
    if (a.split_t) {  // split level: only the in-edges from vertices below split_t (a prefix)
      se = ms_wave_lower_bound(a.cx, sb, se, a.split_t);
      if (se == sb) continue;
    }
    // other chunks' results so far (possibly stale: only less early exit), and
    // on a split level what the light sources pushed
    u64 known = a.accb[v] | (a.split_t ? a.next[v] : 0ull);
    if ((known & need) == need) continue;
    u64 mine = 0ull, posted = 0ull;
    int round = 0;
    for (int base = sb; base < se; base += MS_HU * WAVE) {  // MS_HU rounds of 64 in-edges, loads in flight together
      int u[MS_HU];
#pragma unroll
      for (int r = 0; r < MS_HU; ++r) {
        const int j = base + r * WAVE + lane();
        u[r] = j < se ? a.cx[j] : -1;
      }
      bool hit[MS_HU];
#pragma unroll
      for (int r = 0; r < MS_HU; ++r) hit[r] = ms_probe<SUM, PROBE>(a, s_sum, u[r]);
      u64 f = 0ull;
#pragma unroll
      for (int r = 0; r < MS_HU; ++r)
        if (hit[r]) {
          const u64 w = a.front[u[r]];
          f |= w;
          st.c[C_HITS] += 1;  // a gathered word (zero as well, on paths without the probe)
          st.c[C_HHITS] += 1;
        }
      f = wave_or_u64(f);
      mine |= f & need;
      if (lane() == 0) {
        st.c[C_SCAN] += (u32)min(MS_HU * WAVE, se - base);
        st.c[C_HSCAN] += (u32)min(MS_HU * WAVE, se - base);
      }
      if (((known | mine) & need) == need) break;
      if (++round % MS_POST == 0 && (mine & ~posted)) {
        u64 old = 0ull;
        if (lane() == 0) old = atomicOr(a.accb + v, mine);
        known |= lane_bcast(old, 0);
        posted = mine;
        if (((known | mine) & need) == need) break;
      }
    }
    if (lane() == 0 && (mine & ~posted & ~known)) atomicOr(a.accb + v, mine);
  }
  ms_flush_block<ms_bit(C_SCAN) | ms_bit(C_HITS) | ms_bit(C_HSCAN) | ms_bit(C_HHITS)>(st, a.sh);
}

// Exclusive scans of VPT values per thread at once, in the order
// (slot j, thread t): slot j of thread t gets the sum of every slot j' < j of
// all threads plus slot j of threads < t.  *total gets the sum of all.  Two
// barriers.
template <int VPT>
__device__ __forceinline__ void ms_multi_scan(const int (&x)[VPT], int (&off)[VPT], int *total,
                                              int (*s_w)[BLOCK / WAVE]) {
  const int w = threadIdx.x / WAVE;
  int incl[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    incl[j] = wave_incl_scan(x[j]);
    if (lane() == WAVE - 1) s_w[j][w] = incl[j];
  }
  __syncthreads();
  int run = 0;
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    int before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / WAVE; ++i) {
      const int tw = s_w[j][i];
      before += i < w ? tw : 0;
      all += tw;
    }
    off[j] = run + before + incl[j] - x[j];
    run += all;
  }
  *total = run;
  __syncthreads();
}

// Inclusive segmented OR over the wave: lane l gets the OR of x over the lanes
// l' <= l with key[l'] == key[l], for keys that never decrease from lane to
// lane (a key's lanes are contiguous).  DPP moves instead of LDS permutes:
// shifts by 1, 2, 4 and 8 inside each 16-lane row, then the last lane of row
// 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3; a lane takes a
// moved value only when its key is the lane's own (a lane with no source
// keeps ~key, which never matches).  *tail: the lane is its key's last.
__device__ __forceinline__ u64 ms_seg_or(u64 x, int key, bool *tail) {
  u32 lo = (u32)x, hi = (u32)(x >> 32);
#define MS_SEG_STEP(CTRL, ROWS)                                                       \
  {                                                                                   \
    const int yk = __builtin_amdgcn_update_dpp(~key, key, CTRL, ROWS, 0xf, false);    \
    const u32 yl = (u32)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, ROWS, 0xf, false); \
    const u32 yh = (u32)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, ROWS, 0xf, false); \
    if (yk == key) {                                                                  \
      lo |= yl;                                                                       \
      hi |= yh;                                                                       \
    }                                                                                 \
  }
  MS_SEG_STEP(0x111, 0xf)  // row_shr:1
  MS_SEG_STEP(0x112, 0xf)  // row_shr:2
  MS_SEG_STEP(0x114, 0xf)  // row_shr:4
  MS_SEG_STEP(0x118, 0xf)  // row_shr:8
  MS_SEG_STEP(0x142, 0xa)  // row_bcast:15, rows 1 and 3
  MS_SEG_STEP(0x143, 0xc)  // row_bcast:31, rows 2 and 3
#undef MS_SEG_STEP
  *tail = __builtin_amdgcn_update_dpp(~key, key, 0x130, 0xf, 0xf, false) != key;  // wave_shl:1: lane l + 1's key
  return ((u64)hi << 32) | lo;
}

// Bottom-up, tile part: one workgroup per tile of VPT * BLOCK consecutive
// vertices (slot j of thread t holds vertex tile_base + j * BLOCK + t, so
// every load and store of a slot is coalesced and a wave's slot is one word of
// the bitmaps).  A light vertex's own thread first ORs the frontier words of
// its first MS_HEAD in-edges (bitmap probe first).  The remaining in-edge
// lists of the vertices that still miss lanes are laid end to end (one scan
// over all slots) and walked MS_EPT * BLOCK edges per iteration.  CONSEC
// (sparse frontiers, one round): MS_EPT consecutive edges per thread; the
// thread finds the vertex of its first edge by binary search over the scanned
// offsets in LDS and advances linearly, skips the gathers of a vertex that
// already has all its missing lanes, ORs the gathered words per vertex, and
// posts them with LDS atomics (the last vertex of each thread through one
// segmented scan over the wave).  Otherwise (dense frontiers, capped rounds):
// edge i * BLOCK + t per position, each with its own owner search and
// done-check, one segmented scan per position.  Heavy vertices take the heavy pass's result from accb.  Also
// writes next, the next bitmap and the discoveries, and clears the dead
// frontier buffer.  SPLIT: a split level (MsArgs::split_t).
// At least 5 waves per SIMD: the four-vertex forms fit 96 registers without
// spilling (4 waves at their unconstrained 102-106), and the extra wave hides
// more of the load chain (tile pass 133 -> 126 us per launch); 6 would spill.
template <int VPT, bool SUM, bool CONSEC, bool SPLIT = false, bool PROBE = true>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void k_ms_pull_tile(MsArgs a) {
  constexpr int TV = VPT * BLOCK;
  extern __shared__ u32 s_sum[];
  __shared__ int s_off[TV + 1];
  __shared__ int s_beg[TV];
  __shared__ u64 s_need[TV];
  __shared__ u64 s_acc[TV];
  __shared__ int s_w[VPT][BLOCK / WAVE];
  ms_clear_dead(a);
  ms_stage_summary<SUM>(a, s_sum);
  MsStats st;
  const int t = threadIdx.x;
  const int ngroups = (a.ntiles + VPT - 1) / VPT;
  for (int tile = blockIdx.x; tile < ngroups; tile += gridDim.x) {  // uniform per workgroup
    // VPT consecutive tiles: at most TV vertices, the first a multiple of 64
    const int vb = min(max(a.tstart[tile * VPT], 0), a.n);
    const int ve = min(min(a.tstart[min(tile * VPT + VPT, a.ntiles)], a.n), vb + TV);
    if (vb >= ve) continue;
    u64 vw[VPT], need[VPT], acc[VPT];
    int len[VPT], b[VPT], d[VPT];
    bool heavy[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = vb + j * BLOCK + t;
      vw[j] = v < ve ? a.vis[v] : ~0ull;
      need[j] = a.full & ~vw[j];
      acc[j] = 0ull;
      len[j] = 0;
      b[j] = 0;
      d[j] = 0;
      heavy[j] = false;
    }
    // in-edge offsets (and on a split level what the light sources pushed)
    // for every vertex of the tile, loaded with the visited words rather
    // than after them: the range is read in whole lines either way, and the
    // head loads below wait for one round trip less
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = vb + j * BLOCK + t;
      if (v < ve) {
        b[j] = a.cp[v];
        d[j] = a.cp[v + 1];
        if (SPLIT) acc[j] = a.next[v];
      }
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      if (need[j]) {
        st.c[C_UNVIS] += 1;
        d[j] -= b[j];
        heavy[j] = d[j] > MS_HEAVY;
      } else {
        b[j] = d[j] = 0;
        if (SPLIT) acc[j] = 0ull;
      }
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      if (!need[j]) continue;
      const int v = vb + j * BLOCK + t;
      if (heavy[j]) {
        const u64 h = a.accb[v];
        acc[j] |= h;
        if (h) a.accb[v] = 0ull;  // ready for the next bottom-up level
        continue;
      }
      if (SPLIT && (acc[j] & need[j]) == need[j]) continue;  // covered by the push
      int u[MS_HEAD];
      if (b[j] + MS_HEAD <= a.ncx) {  // the head window lies inside the column array: 16-byte loads
        // (only the pieces that hold list entries); a short list's window runs
        // into the next lists, whose entries are masked off
        const I4u *p = reinterpret_cast<const I4u *>(a.cx + b[j]);
#pragma unroll
        for (int q = 0; q < MS_HEAD / 4; ++q) {
          I4u w = {-1, -1, -1, -1};
          if (4 * q < d[j]) w = p[q];
          u[4 * q] = w.x;
          u[4 * q + 1] = w.y;
          u[4 * q + 2] = w.z;
          u[4 * q + 3] = w.w;
        }
#pragma unroll
        for (int i = 0; i < MS_HEAD; ++i)
          if (i >= d[j]) u[i] = -1;
      } else {
#pragma unroll
        for (int i = 0; i < MS_HEAD; ++i) u[i] = i < d[j] ? a.cx[b[j] + i] : -1;
      }
      bool more = d[j] > MS_HEAD;  // the list goes on past the head
      if (SPLIT) {  // read up to the first in-neighbour >= split_t (pushed instead)
        if (more && u[MS_HEAD - 1] >= a.split_t) more = false;
#pragma unroll
        for (int i = 0; i < MS_HEAD; ++i)
          if (u[i] >= a.split_t) u[i] = -1;
      }
      bool hit[MS_HEAD];
#pragma unroll
      for (int i = 0; i < MS_HEAD; ++i) hit[i] = ms_probe<SUM, PROBE>(a, s_sum, u[i]);
#pragma unroll
      for (int i = 0; i < MS_HEAD; ++i)
        if (hit[i]) {
          const u64 w = a.front[u[i]];
          acc[j] |= w;
          st.c[C_HITS] += 1;
        }
      st.c[C_SCAN] += (u32)min(d[j], MS_HEAD);
      if (more && (acc[j] & need[j]) != need[j]) {
        const int e = SPLIT ? ms_lower_bound(a.cx, b[j] + MS_HEAD, b[j] + d[j], a.split_t) : b[j] + d[j];
        len[j] = e - b[j] - MS_HEAD;
        b[j] += MS_HEAD;
      }
    }
    bool pend = false;
#pragma unroll
    for (int j = 0; j < VPT; ++j) pend |= len[j] > 0;
    // Rounds: each pending vertex walks at most `cap` more in-edges per round
    // (cap grows 4x per round), and vertices whose missing lanes are covered
    // drop out between rounds.  With a sparse frontier few vertices finish
    // early, and the host passes a cap that takes every list in one round.
    for (int cap = a.cap0; __syncthreads_or(pend); cap = cap > (1 << 28) ? cap : cap * 4) {  // uniform
      int take[VPT], off[VPT], total;
#pragma unroll
      for (int j = 0; j < VPT; ++j) take[j] = min(len[j], cap);
      ms_multi_scan(take, off, &total, s_w);
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int l = j * BLOCK + t;
        s_off[l] = off[j];
        s_beg[l] = b[j];
        s_need[l] = need[j];
        s_acc[l] = acc[j];
      }
      if (t == 0) s_off[TV] = total;
      __syncthreads();
      if (CONSEC) {
        for (int c0 = 0; c0 < total; c0 += MS_EPT * BLOCK) {  // uniform per workgroup
          // thread t takes MS_EPT consecutive positions of the laid-out lists:
          // one binary search for the first owner, then a linear advance
          const int e0 = c0 + t * MS_EPT;
          int o = -1, next_off = 0, base_j = 0;
          bool skip = true;
          if (e0 < total) {
            int lo = 0, hi = TV;  // s_off[lo] <= e0 < s_off[hi]
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (s_off[mid] <= e0) lo = mid; else hi = mid;
            }
            o = lo;
            next_off = s_off[o + 1];
            base_j = s_beg[o] - s_off[o];
            const u64 nd = s_need[o];
            skip = (s_acc[o] & nd) == nd;  // lanes already complete: no more gathers for o
          }
          int own[MS_EPT], u[MS_EPT];
          if (o >= 0 && e0 + MS_EPT <= next_off) {
            // all MS_EPT positions in owner o's list: MS_EPT / 4 16-byte loads
            // (4-byte aligned) instead of MS_EPT scalar ones
  #pragma unroll
            for (int i = 0; i < MS_EPT; ++i) own[i] = o;
            if (!skip) {
              const I4u *p = reinterpret_cast<const I4u *>(a.cx + base_j + e0);
  #pragma unroll
              for (int q = 0; q < MS_EPT / 4; ++q) {
                const I4u w = p[q];
                u[4 * q] = w.x;
                u[4 * q + 1] = w.y;
                u[4 * q + 2] = w.z;
                u[4 * q + 3] = w.w;
              }
              st.c[C_SCAN] += MS_EPT;
            } else {
  #pragma unroll
              for (int i = 0; i < MS_EPT; ++i) u[i] = -1;
            }
          } else {
  #pragma unroll
            for (int i = 0; i < MS_EPT; ++i) {
              const int e = e0 + i;
              own[i] = -1;
              u[i] = -1;
              if (o >= 0 && e < total) {
                while (e >= next_off) {  // next owner with edges left (s_off[TV] = total > e)
                  ++o;
                  next_off = s_off[o + 1];
                  base_j = s_beg[o] - s_off[o];
                  const u64 nd = s_need[o];
                  skip = (s_acc[o] & nd) == nd;
                }
                own[i] = o;
                if (!skip) {
                  u[i] = a.cx[base_j + e];
                  st.c[C_SCAN] += 1;
                }
              }
            }
          }
          bool hit[MS_EPT];
  #pragma unroll
          for (int i = 0; i < MS_EPT; ++i) hit[i] = ms_probe<SUM, PROBE>(a, s_sum, u[i]);
          // OR per owner inside the thread; a segment that ends inside the thread
          // is posted directly, the thread's last segment goes through one
          // segmented scan over the wave (equal owners in neighbouring lanes merge)
          u64 run = 0ull;
          int ro = own[0];
  #pragma unroll
          for (int i = 0; i < MS_EPT; ++i) {
            const u64 f = hit[i] ? a.front[u[i]] : 0ull;
            st.c[C_HITS] += hit[i] ? 1 : 0;
            if (own[i] != ro) {
              if (run) atomicOr(&s_acc[ro], run);
              run = 0ull;
              ro = own[i];
            }
            run |= f;
          }
          if (__ballot(run != 0ull)) {
            bool tail;
            run = ms_seg_or(run, ro, &tail);
            if (tail && run) atomicOr(&s_acc[ro], run);
          }
        }
      } else {
        for (int c0 = 0; c0 < total; c0 += MS_EPT * BLOCK) {  // uniform per workgroup
          // position i * BLOCK + t of the batch: one owner search per edge, the
          // done-check per edge, one segmented scan per position
          int own[MS_EPT], u[MS_EPT];
  #pragma unroll
          for (int i = 0; i < MS_EPT; ++i) {
            const int e = c0 + i * BLOCK + t;
            own[i] = -1;
            u[i] = -1;
            if (e < total) {
              int lo = 0, hi = TV;  // s_off[lo] <= e < s_off[hi]
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= e) lo = mid; else hi = mid;
              }
              own[i] = lo;
              const u64 nd = s_need[lo];
              if ((s_acc[lo] & nd) != nd) {
                u[i] = a.cx[s_beg[lo] + (e - s_off[lo])];
                st.c[C_SCAN] += 1;
              }
            }
          }
          bool hit[MS_EPT];
  #pragma unroll
          for (int i = 0; i < MS_EPT; ++i) hit[i] = ms_probe<SUM, PROBE>(a, s_sum, u[i]);
  #pragma unroll
          for (int i = 0; i < MS_EPT; ++i) {
            u64 f = hit[i] ? a.front[u[i]] : 0ull;
            st.c[C_HITS] += hit[i] ? 1 : 0;
            if (__ballot(f != 0ull)) {
              const int oi = own[i];
              bool tail;
              f = ms_seg_or(f, oi, &tail);
              if (tail && f) atomicOr(&s_acc[oi], f);
            }
          }
        }
      }
      __syncthreads();
      pend = false;
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        acc[j] = s_acc[j * BLOCK + t];
        b[j] += take[j];
        len[j] -= take[j];
        if ((acc[j] & need[j]) == need[j]) len[j] = 0;
        pend |= len[j] > 0;
      }
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = vb + j * BLOCK + t;
      u64 nw = 0ull;
      if (v < ve) {
        nw = acc[j] & need[j];
        a.next[v] = nw;
        if (nw) ms_discover(a, v, vw[j], nw, st, d[j]);
        if (heavy[j] && (need[j] & ~nw)) st.c[C_HPEND] += 1;
      }
      const u64 nb = __ballot(nw != 0ull);
      const int w0 = vb + j * BLOCK + (t & ~(WAVE - 1));
      if (lane() == 0 && w0 < ve) a.nbits[w0 / WAVE] = nb;
    }
  }
  ms_flush_block<ms_bit(C_UNVIS) | ms_bit(C_SCAN) | ms_bit(C_HITS) | ms_bit(C_HPEND) | MS_M_FOUND>(st, a.sh);
}

// ------------------------------------------------------------------ push
// ORs lanes m[r] into the next words of v[r] (m[r] = 0: nothing), NR per
// lane at once.  On a sparse level the ORs return the old words, and the
// targets they found zero (first touches: each vertex once per level) are
// appended to the touched list, all NR rounds with one atomic per wave.
// The whole wave calls it.
template <bool SPARSE, int NR>
__device__ __forceinline__ void ms_push_or(const MsArgs &a, const int (&v)[NR], const u64 (&m)[NR]) {
  if (!SPARSE) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (m[r]) atomicOr(a.next + v[r], m[r]);
    return;
  }
  bool first[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) first[r] = m[r] ? atomicOr(a.next + v[r], m[r]) == 0ull : false;
  u64 bm[NR];
  u32 tot = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    bm[r] = __ballot(first[r]);
    tot += (u32)__popcll(bm[r]);
  }
  if (tot == 0u) return;  // uniform
  u32 pos = 0;
  if (lane() == 0) pos = atomicAdd(a.tqn, tot);
  pos = lane_bcast(pos, 0);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (first[r]) a.tq[pos + __popcll(bm[r] & __lanemask_lt())] = v[r];
    pos += (u32)__popcll(bm[r]);
  }
}

// Sparse level: the dead buffer (F_{k-1}'s words) is nonzero only at the
// vertices whose bits the bitmap nbits still holds, so only those words are
// cleared, and the bitmap with them (the sparse update sets F_{k+1}'s bits
// into it).  One wave per 64 bitmap words; the words of one nonzero bitmap
// word go out in one masked store of whole lines.  (On the first level both
// are zero: k_ms_init cleared them.)  The next level's new depth plane, if
// any, is cleared whole.
__device__ __forceinline__ void ms_clear_dead_sparse(const MsArgs &a) {
  const int nwords = (a.n + WAVE - 1) / WAVE;
  const int gw = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE, nwv = gridDim.x * (BLOCK / WAVE);
  for (int w0 = gw * WAVE; w0 < nwords; w0 += nwv * WAVE) {  // uniform per wave
    const int w = w0 + lane();
    const u64 x = w < nwords ? a.nbits[w] : 0ull;
    if (x) a.nbits[w] = 0ull;
    // whole 64-byte lines: each byte of the bitmap word that has a bit set
    // clears its eight words (the others are zero already), so no line is
    // written in part
    u64 y = x | (x >> 1);
    y |= y >> 2;
    y |= y >> 4;
    const u64 lines = (y & 0x0101010101010101ull) * 0xFFull;
    for (u64 nz = __ballot(x != 0ull); nz; nz &= nz - 1ull) {
      const int i = __ffsll((long long)nz) - 1;
      const u64 li = lane_bcast(lines, i);
      if ((li >> lane()) & 1ull) a.dead[(size_t)(w0 + i) * WAVE + lane()] = 0ull;
    }
  }
  if (a.zplane)
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < a.n; i += gridDim.x * BLOCK) a.zplane[i] = 0ull;
}

template <bool SPARSE>
__global__ __launch_bounds__(BLOCK) void k_ms_push(MsArgs a) {
  if (SPARSE)
    ms_clear_dead_sparse(a);
  else
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
    if (fu) {
      b = a.rp[u];
      e = a.rp[u + 1];
      if (e - b > MS_HEAVY) {  // heavy source: its chunks go to k_ms_push_heavy
        e = b;
        atomicOr(a.hsrc, 1u);
      }
    }
    const int d = e - b;  // 0 off the frontier
    {
      int v[MS_T];
      u64 m[MS_T];
#pragma unroll
      for (int t = 0; t < MS_T; ++t) v[t] = t < d ? a.ci[b + t] : -1;
#pragma unroll
      for (int t = 0; t < MS_T; ++t) m[t] = v[t] >= 0 ? fu & ~a.vis[v[t]] : 0ull;
      ms_push_or<SPARSE>(a, v, m);
    }
    st.c[C_SCAN] += (u32)min(d, MS_T);
    const bool pending = d > MS_T;
    b += MS_T;
    u64 pm = __ballot(pending);
    while (pm) {
      const int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      const int vb = lane_bcast(b, l), ve = lane_bcast(e, l);
      const u64 lf = lane_bcast(fu, l);
      for (int base = vb; base < ve; base += MS_HU * WAVE) {  // MS_HU rounds of 64 edges, loads in flight together
        int v[MS_HU];
#pragma unroll
        for (int r = 0; r < MS_HU; ++r) {
          const int j = base + r * WAVE + lane();
          v[r] = j < ve ? a.ci[j] : -1;
        }
        u64 m[MS_HU];
#pragma unroll
        for (int r = 0; r < MS_HU; ++r) m[r] = v[r] >= 0 ? lf & ~a.vis[v[r]] : 0ull;
        ms_push_or<SPARSE>(a, v, m);
      }
      if (lane() == l) st.c[C_SCAN] += (u32)(ve - vb);
    }
  }
  ms_flush_block<ms_bit(C_SCAN)>(st, a.sh);
}

// Split level, push half: the out-lists of the frontier vertices at or above
// push_lo, one wave per list, MS_HU rounds of 64 edges with their loads in
// flight together.  MS_PQ_GRID workgroups; workgroup b takes the bitmap words
// push_lo/64 + b + k * MS_PQ_GRID (interleaved: on a graph numbered by degree
// the busy words sit just above push_lo), 64 words per round, and its waves
// share the round's frontier vertices through an LDS queue.  Light vertices'
// lists start with the same few hubs (ascending lists, hubs first), so edges
// into targets below MS_PQ_HUB are ORed into an LDS copy of those targets'
// `next` words, which each workgroup writes to its row of the staging array
// `hubst` at the end (k_ms_hub_or merges the rows); other targets take one
// global atomic per edge that brings lanes they miss.

__global__ __launch_bounds__(MS_PQ_BLOCK) void k_ms_push_split(MsArgs a) {
  __shared__ u64 s_hub[MS_PQ_HUB];
  __shared__ int s_q[WAVE * WAVE];  // one round: up to 64 words of 64 vertices
  __shared__ int s_qn;
  // the first MS_PQ_HUB targets, hubs or not: on a graph numbered by degree
  // they take the most pushes (the pull that follows starts from these
  // unmasked words and keeps only the lanes each vertex misses)
  const int nh = min(a.n, MS_PQ_HUB);
  for (int i = threadIdx.x; i < nh; i += MS_PQ_BLOCK) s_hub[i] = 0ull;
  MsStats st;
  constexpr int WPB = MS_PQ_BLOCK / WAVE;
  const int wv = threadIdx.x / WAVE;
  const int nwords = (a.n + WAVE - 1) / WAVE, w0 = a.push_lo / WAVE;
  for (long long k0 = 0; w0 + blockIdx.x + k0 * MS_PQ_GRID < nwords; k0 += WAVE) {  // uniform
    if (threadIdx.x == 0) s_qn = 0;
    __syncthreads();
    if (threadIdx.x < WAVE) {
      const long long w = w0 + blockIdx.x + (k0 + threadIdx.x) * MS_PQ_GRID;
      u64 wb = w < nwords ? a.fbits[w] : 0ull;
      if (w == w0) wb &= ~0ull << (a.push_lo % WAVE);  // vertices below push_lo are pulled
      if (wb) {
        int pos = atomicAdd(&s_qn, __popcll(wb));
        for (; wb; wb &= wb - 1ull) s_q[pos++] = (int)w * WAVE + (__ffsll((long long)wb) - 1);
      }
    }
    __syncthreads();
    const int qn = s_qn;
    for (int q = wv; q < qn; q += WPB) {
      const int u = s_q[q];
      const u64 fu = a.front[u];
      const int sb = a.rp[u], se = a.rp[u + 1];
      for (int base = sb; base < se; base += MS_HU * WAVE) {
        int v[MS_HU];
#pragma unroll
        for (int r = 0; r < MS_HU; ++r) {
          const int j = base + r * WAVE + lane();
          v[r] = j < se ? a.ci[j] : -1;
        }
        u64 m[MS_HU];
#pragma unroll
        for (int r = 0; r < MS_HU; ++r) m[r] = v[r] >= nh ? fu & ~a.vis[v[r]] : 0ull;
#pragma unroll
        for (int r = 0; r < MS_HU; ++r) {
          if (v[r] >= 0 && v[r] < nh) atomicOr(&s_hub[v[r]], fu);
          else if (m[r]) atomicOr(a.next + v[r], m[r]);
        }
      }
      if (lane() == 0) {
        st.c[C_SCAN] += (u32)(se - sb);
        st.c[C_PSCAN] += (u32)(se - sb);
        st.c[C_PACT] += 1;
      }
    }
    __syncthreads();  // the queue is refilled next round
  }
  u64 *row = a.hubst + (size_t)blockIdx.x * MS_PQ_HUB;
  for (int i = threadIdx.x; i < nh; i += MS_PQ_BLOCK) row[i] = s_hub[i];
  // counters: one atomic per wave and counter (these workgroups are not BLOCK wide)
  u64 *f = reinterpret_cast<u64 *>(a.sh + (blockIdx.x % NSH));
  const u64 r0 = wave_sum_u64(st.get(C_SCAN)), r1 = wave_sum_u64(st.get(C_PACT));
  if (lane() == 0 && r0) {
    atomicAdd(f + C_SCAN, r0);
    atomicAdd(f + C_PSCAN, r0);
  }
  if (lane() == 0 && r1) atomicAdd(f + C_PACT, r1);
}

// Merges the MS_PQ_GRID staging rows of k_ms_push_split into `next` for the
// targets below min(n, MS_PQ_HUB): thread (i, g) ORs rows
// g * MS_PQ_ROWS .. + MS_PQ_ROWS - 1 of column i.
__global__ __launch_bounds__(BLOCK) void k_ms_hub_or(MsArgs a) {
  const int nh = min(a.n, MS_PQ_HUB);
  const int i = blockIdx.x * BLOCK + threadIdx.x, g = blockIdx.y;
  if (i >= nh) return;
  const u64 *col = a.hubst + (size_t)g * MS_PQ_ROWS * MS_PQ_HUB + i;
  u64 x = 0ull;
#pragma unroll 8
  for (int r = 0; r < MS_PQ_ROWS; ++r) x |= col[(size_t)r * MS_PQ_HUB];
  if (x) atomicOr(a.next + i, x);  // the pull masks these words with the lanes v misses
}
static_assert(MS_PQ_GRID % MS_PQ_ROWS == 0, "staging rows split evenly");

// Top-down, heavy part: one wave per chunk of MS_HCHUNK out-edges of a
// heavy source (out-degree > MS_HEAVY) that is in the frontier, so a hub's
// list is spread over many waves.
template <bool SPARSE>
__global__ __launch_bounds__(BLOCK) void k_ms_push_heavy(MsArgs a) {
  if (__hip_atomic_load(a.hsrc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;  // uniform
  if (a.ochunks < 0) {  // the first level, enqueued before the host read the heavy-list totals
    a.ocount = a.otot[0];
    a.ochunks = a.otot[1];
  }
  MsStats st;
  const int wv = threadIdx.x / WAVE;
  for (int q = blockIdx.x * (BLOCK / WAVE) + wv; q < a.ochunks; q += gridDim.x * (BLOCK / WAVE)) {
    const int i = ms_chunk_owner(a.oq, a.hqcap, a.opre, a.ocount, q);
    const int u = a.ov[i];
    if (!in_front(a.fbits, u)) continue;
    const u64 fu = a.front[u];
    const int sb = a.rp[u] + (q - a.opre[i]) * MS_HCHUNK, se = min(a.rp[u + 1], sb + MS_HCHUNK);
    for (int base = sb; base < se; base += MS_HU * WAVE) {
      int v[MS_HU];
#pragma unroll
      for (int r = 0; r < MS_HU; ++r) {
        const int j = base + r * WAVE + lane();
        v[r] = j < se ? a.ci[j] : -1;
      }
      u64 m[MS_HU];
#pragma unroll
      for (int r = 0; r < MS_HU; ++r) m[r] = v[r] >= 0 ? fu & ~a.vis[v[r]] : 0ull;
      ms_push_or<SPARSE>(a, v, m);
    }
    if (lane() == 0) {
      st.c[C_SCAN] += (u32)(se - sb);
      st.c[C_HSCAN] += (u32)(se - sb);
    }
  }
  ms_flush_block<ms_bit(C_SCAN) | ms_bit(C_HSCAN)>(st, a.sh);
}

// Owner-computes update after a push: F_{k+1}[v] = next[v] (already masked).
__global__ __launch_bounds__(BLOCK) void k_ms_push_update(MsArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.hsrc = 0u;  // k_ms_push_heavy has finished
  if (a.hub_t < 0) a.hub_t = a.otot[0];  // the first level (see MsArgs::hub_t)
  MsStats st;
  for (int base = blockIdx.x * BLOCK; base < a.n; base += gridDim.x * BLOCK) {  // uniform per wave
    const int v = base + threadIdx.x;
    const u64 nw = v < a.n ? a.next[v] : 0ull;
    if (nw) ms_discover(a, v, a.vis[v], nw, st);
    const u64 nb = __ballot(nw != 0ull);
    const int w = (base + (int)(threadIdx.x & ~(WAVE - 1))) / WAVE;
    if (lane() == 0 && w * WAVE < a.n) a.nbits[w] = nb;
  }
  ms_flush_block<MS_M_FOUND>(st, a.sh);
}

// The update of a sparse top-down level: only the touched vertices (each
// listed once, its next word nonzero and already masked); their bits go into
// the bitmap k_ms_push cleared.
__global__ __launch_bounds__(BLOCK) void k_ms_push_update_sparse(MsArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.hsrc = 0u;  // k_ms_push_heavy has finished
  if (a.hub_t < 0) a.hub_t = a.otot[0];  // the first level (see MsArgs::hub_t)
  MsStats st;
  const int cnt = (int)*a.tqn;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < cnt; i += gridDim.x * BLOCK) {
    const int v = a.tq[i];
    ms_discover(a, v, a.vis[v], a.next[v], st);
    atomicOr(a.nbits + (v >> 6), 1ull << (v & 63));
  }
  ms_flush_block<MS_M_FOUND>(st, a.sh);
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

// One output pass over all n columns.
static void launch_ms_out(const MsArgs &a, int flush, hipStream_t s) {
  const int grid = std::min(4096, (a.n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_ms_out, dim3(grid), dim3(BLOCK), 0, s, a, flush);
}


// One bottom-up tile launch: VPT vertices per thread; sum: the frontier is
// tested against its LDS summary first (lds bytes); split: a split level;
// rounds: a dense frontier (capped rounds, gathers without the bitmap probe,
// one owner search per position); otherwise one round of consecutive walks.
template <int VPT>
static void launch_tile(const MsArgs &a, bool sum, bool split, bool rounds, dim3 g, size_t lds, hipStream_t s) {
  if (sum)
    hipLaunchKernelGGL((k_ms_pull_tile<VPT, true, true>), g, dim3(BLOCK), lds, s, a);
  else if (split && rounds)
    hipLaunchKernelGGL((k_ms_pull_tile<VPT, false, false, true, false>), g, dim3(BLOCK), 0, s, a);
  else if (split)
    hipLaunchKernelGGL((k_ms_pull_tile<VPT, false, true, true, false>), g, dim3(BLOCK), 0, s, a);
  else if (rounds)
    hipLaunchKernelGGL((k_ms_pull_tile<VPT, false, false, false, false>), g, dim3(BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((k_ms_pull_tile<VPT, false, true>), g, dim3(BLOCK), 0, s, a);
}

// ------------------------------------------------------------ tuning
// Configurations bfs_multi_autotune found, per graph (array addresses, sizes
// and the degree-order flag); bfs_multi uses one when the caller passes none.
// Only the time depends on it, so an entry left from a freed graph whose
// addresses are reused costs speed, never correctness.
struct MsTuneKey {
  const void *rp, *ci, *cp, *cx;
  int n, nnz, hub;
  bool operator==(const MsTuneKey &o) const {
    return rp == o.rp && ci == o.ci && cp == o.cp && cx == o.cx && n == o.n && nnz == o.nnz && hub == o.hub;
  }
};
static std::mutex g_tune_mu;
static std::vector<std::pair<MsTuneKey, MsTune>> g_tuned;  // most recent last, at most 64

static MsTuneKey ms_tune_key(const bfs_graph *g, int flags) {
  return MsTuneKey{g->row_ptr, g->col_idx, g->csc_ptr, g->csc_idx, g->n, g->nnz, (flags & BFS_F_HUB_ORDER) ? 1 : 0};
}

static int ms_tune_from(const bfs_multi_config &c, MsTune *t) {
  MsTune d;
  const auto vpt_ok = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4; };
  if (c.wide_ratio < 0 || !vpt_ok(c.split_vpt) || !vpt_ok(c.wide_vpt) || !vpt_ok(c.narrow_vpt) || c.cap0 < 0 ||
      (c.tile_alpha != 0 && (c.tile_alpha < MS_TALPHA_MIN || c.tile_alpha > MS_TALPHA_MAX)) || c.alpha < 0 ||
      c.split_lout < 0) {
    set_error("bfs_multi_config: wide_ratio, cap0, alpha and split_lout must be >= 0, split_vpt, wide_vpt and "
              "narrow_vpt 0, 1, 2 or 4, tile_alpha 0 or in [%d, %d]",
              MS_TALPHA_MIN, MS_TALPHA_MAX);
    return BFS_EINVAL;
  }
  t->wide_ratio = c.wide_ratio ? c.wide_ratio : d.wide_ratio;
  t->split_vpt = c.split_vpt ? c.split_vpt : d.split_vpt;
  t->cap0 = c.cap0 ? c.cap0 : d.cap0;
  t->talpha = c.tile_alpha ? c.tile_alpha : d.talpha;
  t->alpha = c.alpha ? c.alpha : d.alpha;
  t->split_lout = c.split_lout ? c.split_lout : d.split_lout;
  t->wide_vpt = c.wide_vpt ? c.wide_vpt : d.wide_vpt;
  t->narrow_vpt = c.narrow_vpt ? c.narrow_vpt : d.narrow_vpt;
  return BFS_OK;
}

static bfs_multi_config ms_config_of(const MsTune &t) {
  bfs_multi_config c;
  c.wide_ratio = t.wide_ratio;
  c.split_vpt = t.split_vpt;
  c.cap0 = t.cap0;
  c.tile_alpha = t.talpha;
  c.alpha = t.alpha;
  c.split_lout = t.split_lout;
  c.wide_vpt = t.wide_vpt;
  c.narrow_vpt = t.narrow_vpt;
  return c;
}

// The configuration of one call: the caller's, else the stored one for the
// graph, else the defaults.
static int ms_resolve_tune(const bfs_graph *g, const bfs_options *opt, MsTune *t) {
  if (opt && opt->multi_config) return ms_tune_from(*opt->multi_config, t);
  *t = MsTune();
  const MsTuneKey key = ms_tune_key(g, opt ? opt->flags : 0);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto &e : g_tuned)
    if (e.first == key) *t = e.second;
  return BFS_OK;
}

static void ms_store_tune(const bfs_graph *g, int flags, const MsTune &t) {
  const MsTuneKey key = ms_tune_key(g, flags);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (size_t i = 0; i < g_tuned.size(); ++i)
    if (g_tuned[i].first == key) {
      g_tuned.erase(g_tuned.begin() + (long)i);
      break;
    }
  if (g_tuned.size() >= 64) g_tuned.erase(g_tuned.begin());
  g_tuned.push_back({key, t});
}

}  // namespace bfs

using namespace bfs;

extern "C" int bfs_multi(const bfs_graph *g, const int32_t *sources, int32_t k, int32_t *levels,
                         const bfs_options *opt, bfs_stats *st, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!g || g->n <= 0 || g->nnz < 0 || !g->row_ptr || (!g->col_idx && g->nnz > 0) || !sources || !levels || k < 1) {
    set_error("bfs_multi: invalid argument (null pointer, n <= 0, nnz < 0 or k < 1)");
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
  MsTune tune;
  rc = ms_resolve_tune(g, opt, &tune);
  if (rc) return rc;
  const MsCarve W = ms_carve(reinterpret_cast<uintptr_t>(wsp), n);
  u64 *const *fr = W.fr;
  MsCtr *sh = W.sh;
  int *src_dev = W.src;
  HostCtx &hc = host_ctx();
  const int grid_v = std::min(4096, (n + BLOCK - 1) / BLOCK);
  const int grid_w = std::min(4096, ((n + WAVE - 1) / WAVE + 3) / 4);
  // heavy in-degree vertices and their chunk prefix (read back with the first group's sync)
  const int nbh = (n + MS_HB - 1) / MS_HB;
  int *htot_dev = src_dev + 192;
  // k_ms_seed posts the totals and the sources' degrees here (coherent host memory)
  int *post_host = reinterpret_cast<int *>(hc.pinned_u64 + 64);
  u64 *post_seq = hc.pinned_u64 + 200;
  const int *htot_host = post_host;
  const int *deg_host = post_host + 64;
  // with the bottom-up tiles (their count in htot[4])
  hipLaunchKernelGGL(k_ms_heavy_count, dim3(nbh), dim3(BLOCK), 0, s, g->csc_ptr, n, W.bcnt, W.bchk, W.bwt,
                     tune.talpha);
  hipLaunchKernelGGL(k_ms_heavy_scan, dim3(1), dim3(BLOCK), 0, s, nbh, W.bcnt, W.bchk, htot_dev, W.bwt,
                     htot_dev + 4, tune.talpha);
  const int hqcap = (int)ms_hq_cap(n);
  hipLaunchKernelGGL(k_ms_heavy_write, dim3(nbh), dim3(BLOCK), 0, s, g->csc_ptr, n, W.bcnt, W.bchk, W.hv, W.hpre,
                     W.hq, hqcap, W.accb, htot_dev, (const long long *)W.bwt, W.tstart, (const int *)(htot_dev + 4),
                     tune.talpha);
  // the same over out-degrees for the top-down step (a symmetric graph passes one array twice)
  if (g->row_ptr != g->csc_ptr) {
    hipLaunchKernelGGL(k_ms_heavy_count, dim3(nbh), dim3(BLOCK), 0, s, g->row_ptr, n, W.bcnt, W.bchk,
                       (long long *)nullptr, tune.talpha);
    hipLaunchKernelGGL(k_ms_heavy_scan, dim3(1), dim3(BLOCK), 0, s, nbh, W.bcnt, W.bchk, htot_dev + 2,
                       (long long *)nullptr, (int *)nullptr, tune.talpha);
    hipLaunchKernelGGL(k_ms_heavy_write, dim3(nbh), dim3(BLOCK), 0, s, g->row_ptr, n, W.bcnt, W.bchk, W.ov, W.opre,
                       W.oq, hqcap, (u64 *)nullptr, htot_dev + 2, (const long long *)nullptr, (int *)nullptr,
                       (const int *)nullptr, tune.talpha);
  }
  BFS_HIP(hipGetLastError());
  long long reached = 0, comp = 0;
  int max_levels = 0, syncs = 0;
  const int flags = opt ? opt->flags : 0;
  const bool rec =
      st && (flags & (BFS_F_LEVEL_STATS | BFS_F_LEVEL_TIMING | BFS_F_MAIN_TIMING)) && st->level_capacity > 0;
  const bool timing = rec && (flags & BFS_F_LEVEL_TIMING);             // all four events per level
  const bool mtiming = rec && (flags & (BFS_F_LEVEL_TIMING | BFS_F_MAIN_TIMING));  // main kernel's two
  int recorded = 0;
  // level timing: the entry whose events are still to be read (-1: none)
  int tslot = 0, pend_r = -1, pend_slot = 0;
  auto resolve_timing = [&]() -> int {
    if (pend_r < 0) return BFS_OK;
    const hipEvent_t *P = hc.lev_ev + 4 * (pend_slot % 16);
    float ms = 0.f;
    // the level's post can be seen before the runtime has marked its events done
    if (st->level_ms_main) {
      BFS_HIP(hipEventSynchronize(P[2]));
      BFS_HIP(hipEventElapsedTime(&ms, P[1], P[2]));
      st->level_ms_main[pend_r] = ms;
    }
    if (st->level_ms && timing) {
      BFS_HIP(hipEventSynchronize(P[3]));
      BFS_HIP(hipEventElapsedTime(&ms, P[0], P[3]));
      st->level_ms[pend_r] = ms;
    }
    pend_r = -1;
    return BFS_OK;
  };
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
    a.ncx = g->nnz;
    a.sym = g->row_ptr == g->csc_ptr ? 1 : 0;
    a.vis = W.vis;
    a.planes = W.planes;
    a.flushed = W.flushed;
    a.accb = W.accb;
    a.hv = W.hv;
    a.hpre = W.hpre;
    a.tstart = W.tstart;
    a.fsum = W.fsum;
    a.sshift = 4;
    while (((long long)n >> a.sshift) > (long long)MS_SUM_WORDS * 32) ++a.sshift;
    a.levels = levels + (size_t)g0 * n;
    a.vmap = opt ? opt->vertex_map : nullptr;
    a.hsrc = reinterpret_cast<u32 *>(src_dev + 200);
    a.tqn = reinterpret_cast<u32 *>(src_dev + 203);
    a.tq = W.tq;
    a.sparse = 0;
    a.hubst = W.hubst;
    a.sh = sh;
    a.base = 0;
    a.np = 2;  // planes 0 and 1 are cleared by k_ms_init
    a.nflush = 0;
    hipLaunchKernelGGL(k_ms_init, dim3(grid_v), dim3(BLOCK), 0, s, a, fr[0], fr[1], fr[2], W.fb[0], W.fb[1]);
    // sources by value; the seed kernel posts the counts of F_0 for the
    // direction rule (distinct source vertices and their degrees) and the
    // heavy-list and tile totals, which the host polls for
    MsSources sv;
    for (int i = 0; i < 64; ++i) sv.v[i] = i < L ? sources[g0 + i] : 0;
    const u64 seed_seq = ++hc.seq;
    hipLaunchKernelGGL(k_ms_seed, dim3(1), dim3(64), 0, s, a, sv, fr[0], W.fb[0], (const int *)htot_dev, post_host,
                       post_seq, seed_seq);
    BFS_HIP(hipGetLastError());
    // split id: vertices below it are pulled on a split bottom-up level, the
    // frontier vertices at or above it push (options.hub_split > 0: that id on
    // every bottom-up level; 0: on a graph numbered by decreasing degree, its
    // heavy out-degree vertices, where the cost rule below picks it; < 0: never)
    const int hub_req = opt ? opt->hub_split : 0;
    const bool hub_auto = hub_req == 0 && (flags & BFS_F_HUB_ORDER);
    a.push_lo = 0;
    a.split_t = 0;
    const bool sym = g->row_ptr == g->csc_ptr;
    a.ov = sym ? W.hv : W.ov;
    a.opre = sym ? W.hpre : W.opre;
    a.hq = W.hq;
    a.oq = sym ? W.hq : W.oq;
    a.hqcap = hqcap;
    a.otot = sym ? htot_dev : htot_dev + 2;
    long long nf = 0, ef = 0, src_comp = 0;
    // What the seed kernel posted: the heavy-list and tile totals, and the
    // count and out-edges of F_0 for the direction rule.
    auto take_seed = [&]() {
      a.hcount = htot_host[0];
      a.hchunks = htot_host[1];
      a.ntiles = htot_host[4];
      a.ocount = sym ? a.hcount : htot_host[2];
      a.ochunks = sym ? a.hchunks : htot_host[3];
      a.hub_t = hub_req > 0 ? std::min(hub_req, n) : hub_auto ? a.ocount : 0;
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
    };
    // Except when every level is bottom-up, the first level (a frontier of at
    // most 64 sources) is top-down: it is enqueued at once, without waiting
    // for the seed's post, which the host reads with that level's counters.
    bool seed_read = mode == BFS_V_PULL_B;
    if (seed_read) {
      rc = wait_posted(post_seq, seed_seq, s);
      if (rc) return rc;
      take_seed();
    } else {
      a.hcount = a.hchunks = a.ntiles = 0;  // not used by a top-down level
      a.ocount = a.ochunks = -1;
      a.hub_t = hub_req > 0 ? std::min(hub_req, n) : hub_auto ? -1 : 0;
    }
    long long eu = g->nnz;  // in-edges of vertices still missing some lane
    long long lout = ef;    // out-edges of the frontier vertices at or above hub_t (level 0: an upper bound)
    reached += L;
    int msdir = 0;
    long long prev_nf = -1;
    bool heavy_done = false;  // after a bottom-up level left no heavy vertex missing a lane
    int lev = 0;
    for (;;) {
      int dir;
      if (mode == BFS_V_PUSH_Q_THREAD || mode == BFS_V_PUSH_Q_BLOCK || mode == BFS_V_PUSH_Q_MERGE || !seed_read)
        dir = 0;
      else if (mode == BFS_V_PULL_B)
        dir = 1;
      else {
        // Direction rule for bit-packed lanes: a bottom-up step exits early
        // only once every lane a vertex misses is found, so it costs close to
        // all in-edges of the vertices still missing a lane (eu) plus a pass
        // over all n vertices; top-down costs the frontier's out-edges (ef),
        // one atomic each.  Bottom-up when ef > eu / alpha and ef > n / 8;
        // back to top-down under Beamer's beta test.
        if (msdir == 0) {
          if (ef * tune.alpha > eu && ef * 8 > (long long)n) msdir = 1;
        } else if (nf * HeuristicState::kBeta < (long long)n && prev_nf >= 0 && nf < prev_nf) {
          msdir = 0;
        }
        prev_nf = nf;
        dir = msdir;
      }
      // relative depth of this step's discoveries; a full window is written out first
      if (lev + 1 - a.base >= (1 << MS_PLANES)) {
        launch_ms_out(a, 1, s);
        ++a.nflush;
        a.base = lev;
        a.np = 0;
      }
      a.rel = lev + 1 - a.base;
      while ((a.rel >> a.np) != 0) {  // a plane not zeroed ahead (window start): zero it now
        hipLaunchKernelGGL(k_ms_fill, dim3(grid_v), dim3(BLOCK), 0, s, a.planes + (size_t)a.np * n, n);
        ++a.np;
      }
      // the next level stores relative depth rel + 1: if that needs a new plane,
      // this level's step kernels zero it (they clear the dead buffer anyway)
      a.zplane = nullptr;
      if (((a.rel + 1) >> a.np) != 0 && a.np < MS_PLANES) {
        a.zplane = a.planes + (size_t)a.np * n;
        ++a.np;
      }
      a.k = lev;
      a.sparse = 0;
      a.front = fr[lev % 3];
      a.next = fr[(lev + 1) % 3];
      a.dead = fr[(lev + 2) % 3];
      a.fbits = W.fb[lev & 1];
      a.nbits = W.fb[(lev + 1) & 1];
      // timing: four events per level from a ring of 16 sets (level start,
      // main kernel start and end, level end); read after the next level is
      // enqueued, off the path between levels
      hipEvent_t *E = hc.lev_ev + 4 * (tslot % 16);
      if (timing) BFS_HIP(hipEventRecord(E[0], s));
      // Split bottom-up level (see MsArgs::split_t): where the frontier is sparse
      // (no early exits expected, so the plain step reads every in-edge of the
      // vertices missing a lane) and the light frontier vertices' out-edges,
      // one atomic each, cost less than the in-edges skipped.
      const bool split =
          dir == 1 && a.hub_t > 0 && (hub_req > 0 || (ef * 4 <= eu && lout * (long long)tune.split_lout < eu));
      if (dir == 1) {
        // early exits pay for extra rounds only when the frontier carries a
        // large share of the remaining in-edges
        a.cap0 = ef * 4 > eu ? tune.cap0 : (1 << 30);
        if (split) {
          // the light sources push first; the tile kernel clears the dead buffer
          MsArgs ap = a;
          ap.dead = nullptr;
          ap.zplane = nullptr;
          ap.push_lo = a.hub_t;
          hipLaunchKernelGGL(k_ms_push_split, dim3(MS_PQ_GRID), dim3(MS_PQ_BLOCK), 0, s, ap);
          hipLaunchKernelGGL(k_ms_hub_or, dim3((std::min(a.n, MS_PQ_HUB) + BLOCK - 1) / BLOCK,
                                               MS_PQ_GRID / MS_PQ_ROWS), dim3(BLOCK), 0, s, ap);
          a.split_t = a.hub_t;
        }
        // a sparse frontier is tested against its LDS summary first: most
        // in-neighbours are rejected without touching the bitmap
        // (the heavy pass, which exits early per chunk, gains from it only
        // at much lower densities than the tile pass).  Not on a graph
        // renumbered by degree: there most in-edges come from the first few
        // hundred KB of bitmap, which stay in cache, and the 32 KB of LDS per
        // workgroup would cost more in occupancy than the filter saves.
        const bool filt = !(flags & BFS_F_HUB_ORDER) && !split;
        const bool sum = filt && (nf << a.sshift) * 8 < (long long)n;
        const bool hsum = filt && (nf << a.sshift) * 64 < (long long)n;
        if (sum)
          hipLaunchKernelGGL(k_ms_summary, dim3(MS_SUM_WORDS / BLOCK), dim3(BLOCK), 0, s, (const u64 *)a.fbits,
                             (n + 63) / 64, W.fsum, a.sshift);
        const size_t lds = sum ? MS_SUM_WORDS * sizeof(u32) : 0;
        if (a.hchunks > 0 && !heavy_done) {
          const int gh = std::min(hsum ? MS_SUM_GRID : 4096, (a.hchunks + 3) / 4);
          if (hsum) {
            hipLaunchKernelGGL(k_ms_pull_heavy<true>, dim3(gh), dim3(BLOCK), lds, s, a, 0);
          } else if (ef * 4 > eu) {  // dense frontier (see `rounds`): first chunks first, no bitmap probe
            const int g1 = std::min(4096, (a.hcount + 3) / 4);
            hipLaunchKernelGGL((k_ms_pull_heavy<false, false>), dim3(g1), dim3(BLOCK), 0, s, a, 1);
            hipLaunchKernelGGL((k_ms_pull_heavy<false, false>), dim3(gh), dim3(BLOCK), 0, s, a, 2);
          } else if (split) {  // gathers of hub words without the probe
            hipLaunchKernelGGL((k_ms_pull_heavy<false, false>), dim3(gh), dim3(BLOCK), 0, s, a, 0);
          } else {
            hipLaunchKernelGGL(k_ms_pull_heavy<false>, dim3(gh), dim3(BLOCK), 0, s, a, 0);
          }
        }
        // one vertex per thread while many in-edges remain to be scanned (more
        // workgroups in flight); four when few do, and on split levels, which
        // read only the hubs' part of each list (fixed costs amortised, and
        // four vertices' loads in flight per thread)
        if (mtiming) BFS_HIP(hipEventRecord(E[1], s));
        const bool rounds = a.cap0 < (1 << 30);  // dense frontier: per-position walk
        const int vpt = split ? tune.split_vpt : eu > (long long)tune.wide_ratio * n ? tune.wide_vpt : tune.narrow_vpt;
        const int gtiles = std::min(65536, (a.ntiles + vpt - 1) / vpt);
        const dim3 gt(sum ? std::min(gtiles, MS_SUM_GRID) : gtiles);
        switch (vpt) {
          case 1: launch_tile<1>(a, sum, split, rounds, gt, lds, s); break;
          case 2: launch_tile<2>(a, sum, split, rounds, gt, lds, s); break;
          default: launch_tile<4>(a, sum, split, rounds, gt, lds, s); break;
        }
        if (mtiming) BFS_HIP(hipEventRecord(E[2], s));
        a.split_t = 0;
      } else {
        // Sparse level (few frontier out-edges, or the first level, whose
        // counts the host reads with its totals): the vertices it reaches are
        // listed and only they are updated, and the dead buffer is cleared at
        // F_{k-1}'s vertices only, instead of passes over all n words.
        const bool sparse = !seed_read || ef * 8 < (long long)n;
        a.sparse = sparse ? 1 : 0;
        if (mtiming) BFS_HIP(hipEventRecord(E[1], s));
        if (sparse)
          hipLaunchKernelGGL(k_ms_push<true>, dim3(grid_w), dim3(BLOCK), 0, s, a);
        else
          hipLaunchKernelGGL(k_ms_push<false>, dim3(grid_w), dim3(BLOCK), 0, s, a);
        if (mtiming) BFS_HIP(hipEventRecord(E[2], s));
        // chunk count not read back yet (first level): a grid for any graph; the kernel
        // reads the count, and returns at once unless a heavy source is in the frontier
        const long long och = a.ochunks >= 0 ? a.ochunks : 2 * (long long)g->nnz / MS_HCHUNK + 1;
        const dim3 gph((unsigned)std::min<long long>(4096, (och + 3) / 4));
        if (och > 0 && sparse)
          hipLaunchKernelGGL(k_ms_push_heavy<true>, gph, dim3(BLOCK), 0, s, a);
        else if (och > 0)
          hipLaunchKernelGGL(k_ms_push_heavy<false>, gph, dim3(BLOCK), 0, s, a);
        if (sparse) {  // at most ef vertices touched (any number on the first level)
          const long long gu = seed_read ? std::max(1LL, std::min(4096LL, (ef + BLOCK - 1) / BLOCK)) : 1024LL;
          hipLaunchKernelGGL(k_ms_push_update_sparse, dim3((unsigned)gu), dim3(BLOCK), 0, s, a);
        } else {
          hipLaunchKernelGGL(k_ms_push_update, dim3(grid_v), dim3(BLOCK), 0, s, a);
        }
      }
      if (timing) BFS_HIP(hipEventRecord(E[3], s));
      MsCtr *tot_host = reinterpret_cast<MsCtr *>(hc.pinned);
      const u64 seq = ++hc.seq;
      hipLaunchKernelGGL(k_ms_finish, dim3(1), dim3(NSH), 0, s, sh, tot_host, seq, a.sparse ? a.tqn : nullptr);
      BFS_HIP(hipGetLastError());
      rc = resolve_timing();  // the previous level's events, while this one runs
      if (rc) return rc;
      rc = wait_posted(&tot_host->seq, seq, s);
      if (rc) return rc;
      ++syncs;
      MsCtr c;
      memcpy(&c, hc.pinned, sizeof(c));
      if (!seed_read) {  // the seed kernel's post is complete: it ran before this level
        take_seed();
        prev_nf = nf;  // the direction rule's state after a first level it did not choose
        seed_read = true;
      }
      if (rec && recorded < st->level_capacity) {
        // entry: one level of one group; variant 6 = bottom-up, 0 = top-down
        const int r = recorded++;
        if (st->level_variant)
          st->level_variant[r] = split ? BFS_MS_SPLIT : dir == 1 ? BFS_V_PULL_B : BFS_V_PUSH_Q_THREAD;
        if (st->level_frontier) st->level_frontier[r] = nf;
        if (st->level_frontier_edges) st->level_frontier_edges[r] = ef;
        if (st->level_unvisited) st->level_unvisited[r] = (long long)c.unvis;
        if (st->level_unvisited_edges) st->level_unvisited_edges[r] = eu;
        if (st->level_scanned) st->level_scanned[r] = (long long)c.scanned;
        if (st->level_next) st->level_next[r] = (long long)c.newbits;
        if (st->level_frontier_ld) st->level_frontier_ld[r] = (long long)c.active;
        if (st->level_frontier_ld2) st->level_frontier_ld2[r] = (long long)c.hits;
        if (st->level_scanned_aux) st->level_scanned_aux[r] = (long long)c.hscanned;
        if (st->level_hits_aux) st->level_hits_aux[r] = (long long)c.hhits;
        if (st->level_scanned_push) st->level_scanned_push[r] = (long long)c.pscan;
        if (st->level_push_sources) st->level_push_sources[r] = (long long)c.pact;
        if (st->level_ms_main) st->level_ms_main[r] = 0.f;
        if (st->level_ms) st->level_ms[r] = 0.f;
        if (mtiming) pend_r = r, pend_slot = tslot;
      }
      ++tslot;
      if (dir == 1 && c.hpend == 0) heavy_done = true;  // visited words only grow
      ++lev;
      if (c.newbits == 0) break;
      reached += (long long)c.newbits;
      comp += (long long)c.comp_edges;
      nf = (long long)c.active;
      ef = (long long)c.active_out;
      lout = (long long)c.lout;
      eu -= (long long)c.done_in;
      if (lev > n + 1) {
        set_error("bfs_multi: level loop did not converge");
        return BFS_ELEVELCAP;
      }
    }
    comp += src_comp;  // each lane's source belongs to its component
    launch_ms_out(a, 0, s);
    BFS_HIP(hipGetLastError());
    max_levels = std::max(max_levels, lev);
    rc = resolve_timing();
    if (rc) return rc;
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

extern "C" int bfs_multi_autotune(const bfs_graph *g, const int32_t *sources, int32_t k, int32_t *levels,
                                  const bfs_options *opt, bfs_multi_config *best, float *ms_best, void *stream) {
  if (!best) {
    set_error("bfs_multi_autotune: best is NULL");
    return BFS_EINVAL;
  }
  bfs_options o;
  if (opt) {
    o = *opt;
  } else {
    memset(&o, 0, sizeof(o));
    o.variant = BFS_AUTO_HEURISTIC;
  }
  o.flags &= ~(BFS_F_LEVEL_STATS | BFS_F_LEVEL_TIMING | BFS_F_MAIN_TIMING);
  MsTune cur;
  if (opt && opt->multi_config) {
    const int rc = ms_tune_from(*opt->multi_config, &cur);
    if (rc) return rc;
  }
  // device time of one configuration: best of two runs (the first also
  // warms the caches and the library's workspace)
  auto time_of = [&](const MsTune &t, float *ms) -> int {
    const bfs_multi_config c = ms_config_of(t);
    o.multi_config = &c;
    float bestv = 0.f;
    for (int r = 0; r < 2; ++r) {
      bfs_stats st;
      memset(&st, 0, sizeof(st));
      const int rc = bfs_multi(g, sources, k, levels, &o, &st, stream);
      if (rc) return rc;
      if (r == 0 || st.elapsed_ms < bestv) bestv = st.elapsed_ms;
    }
    *ms = bestv;
    return BFS_OK;
  };
  float cur_ms = 0.f;
  int rc = time_of(cur, &cur_ms);
  if (rc) return rc;
  // one field at a time, each over its candidates, keeping the fastest
  static const int wide_c[] = {2, 4, 8, 16, 64, 1 << 20};
  static const int vpt_c[] = {1, 2, 4};
  static const int cap_c[] = {16, 32, 64, 128};
  static const int talpha_c[] = {32, 64, 128};
  static const int alpha_c[] = {4, 7, 14};
  static const int lout_c[] = {4, 16, 64};
  struct Field {
    int MsTune::*f;
    const int *c;
    int nc;
  };
  const Field fields[] = {{&MsTune::wide_ratio, wide_c, 6}, {&MsTune::wide_vpt, vpt_c, 3},
                          {&MsTune::narrow_vpt, vpt_c, 3},  {&MsTune::split_vpt, vpt_c, 3},
                          {&MsTune::cap0, cap_c, 4},        {&MsTune::talpha, talpha_c, 3},
                          {&MsTune::alpha, alpha_c, 3},     {&MsTune::split_lout, lout_c, 3}};
  for (const Field &fd : fields) {
    for (int i = 0; i < fd.nc; ++i) {
      if (cur.*(fd.f) == fd.c[i]) continue;
      MsTune t = cur;
      t.*(fd.f) = fd.c[i];
      float ms = 0.f;
      rc = time_of(t, &ms);
      if (rc) return rc;
      if (ms < 0.99f * cur_ms) {  // a clear gain only: run-to-run noise does not move the choice
        cur = t;
        cur_ms = ms;
      }
    }
  }
  ms_store_tune(g, o.flags, cur);
  *best = ms_config_of(cur);
  if (ms_best) *ms_best = cur_ms;
  return BFS_OK;
}
