/*
 * bfs_eeds.h -- C ABI of the MI355X (gfx950) BFS level-step library.
 *
 * The library computes breadth-first-search depths as the paper's EDGE BFS
 * cascade defines them (Cascade 1, Sec. "Expressing BFS with EDGE"): from
 * F_0 = {s}, P_0 = {s}, every level computes
 *     F_{i+1}[d] = OR_s (F_i[s] AND G[s,d]) AND NOT P_i[d]      (Eq. advance)
 *     P_{i+1}    = P_i OR F_{i+1}                                (Eq. update)
 * and records depth i+1 for every d in F_{i+1}; the search stops when
 * F_{i+1} is empty.  Depths are the minimum number of hops from the source
 * (the problem statement of the same section).  Every variant below reaches
 * exactly the same depths; the paper's design-space sections (Sec. "The
 * Einsum-Enabled Design Space", Table 3) describe the transformations that
 * separate them.
 *
 * Conventions shared by every entry point
 *   - Graph arrays, depth/parent outputs and workspaces are DEVICE pointers
 *     allocated and owned by the caller; the library never keeps them past
 *     the call.  Arrays named *_host are host pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call
 *     enqueues its work on that stream and returns after it has completed,
 *     so outputs and statistics are valid on return.
 *   - Return value 0 on success or a negative BFS_E* code; nothing throws.
 *     bfs_last_error() gives a thread-local message for the last failure.
 *   - Depth -1 and parent -1 mean "unreached" (the paper's empty value,
 *     infinity, Cascade 1 tensor declarations).  parents[source] = source.
 *   - A vertex id is int32; CSR offsets are int32, so nnz < 2^31.
 *   - Calls on different streams are independent when each has its own
 *     workspace; two calls sharing a workspace must not overlap.
 */
#ifndef BFS_EEDS_H
#define BFS_EEDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define BFS_OK 0
#define BFS_EINVAL (-1)     /* null pointer, n <= 0, source out of range, bad count or id */
#define BFS_EGRAPH (-2)     /* BFS_F_VALIDATE set and the CSR/CSC is malformed */
#define BFS_EWORKSPACE (-3) /* workspace smaller than bfs_workspace_size() */
#define BFS_EHIP (-4)       /* a HIP runtime call failed (detail in bfs_last_error) */
#define BFS_ENOSEL (-5)     /* learned mode with BFS_F_STRICT_SELECTOR and no weights */
#define BFS_ELEVELCAP (-6)  /* the level loop hit options.max_levels */
#define BFS_ENOTSUP (-7)    /* requested variant needs CSC arrays that were not given */
#define BFS_EFILE (-8)      /* selector weights file missing, short or malformed */

const char *bfs_strerror(int code);
const char *bfs_last_error(void);
int bfs_version(void);

/* -------------------------------------------------------------- variants
 * Fixed variants (one per level; each is a point of the paper's design space):
 *  PUSH_Q_THREAD   top-down over CSR, queue frontier, one lane per frontier
 *                  vertex, atomic visited claim            (Table 3, variant 2)
 *  PUSH_Q_BLOCK    top-down, queue, a workgroup flattens the edges of 256
 *                  frontier vertices and splits them evenly over its lanes;
 *                  vertices above a degree threshold are split across the whole
 *                  grid                                    (Table 3, variant 1)
 *  PUSH_Q_MERGE    top-down, queue, merge-path: the frontier's edge space is
 *                  flattened by a device-wide degree scan and cut into equal
 *                  tiles                                   (Table 3, variant 3)
 *  PUSH_B_ATOMIC   top-down, bitmap frontier in, atomic claim (Table 3, variant 10)
 *  PUSH_B_NOATOMIC top-down, bitmap frontier, explicit visited mask, no atomics:
 *                  depth stores are idempotent and the visited/frontier
 *                  bitmaps are rebuilt by an owner-computes pass
 *                                                 (Table 3, variants 12/21/24)
 *  PUSH_Q_NOATOMIC as above with a queue frontier in   (Table 3, variant 21)
 *  PULL_B          bottom-up over CSC with early exit: each unvisited vertex
 *                  scans its in-neighbours and stops at the first frontier
 *                  member (Sec. "From Push to Pull BFS": reassociate, commute,
 *                  reassociate, loop order d -> s)
 *  PULL_VIS        bottom-up with the visited set as the frontier (Table 3,
 *                  variant 25): an unvisited vertex's reached in-neighbours
 *                  all lie at the current depth, so the visited bitmap (bits
 *                  of never-reachable vertices told apart by their depth, -1)
 *                  serves as the frontier; new bits are merged after the step
 *  PUSH_P3         top-down with three visited arrays (Table 3, variant 26):
 *                  no frontier array, F_k = P_k AND NOT P_{k-1}; atomic-free
 *                  expansion as PUSH_B_NOATOMIC, and the owner-computes update
 *                  keeps P_k as the next level's P_{k-1}
 *  PUSH_Q_FILTER   top-down, queue, advance before the depth update (Table 3,
 *                  variant 13): a merge-path pass writes every out-neighbour of
 *                  F_k with its source to a temporary list (no visited test, no
 *                  atomics), then a filter pass claims each entry as the atomic
 *                  push does; the list holds tmp_entries(n) entries (n clamped
 *                  to [2^16, 2^22]), larger frontiers go in chunks
 *  PUSH_B_FILTER   the same with a bitmap frontier (Table 3, variant 14): the
 *                  edge space is flattened word by word over the bitmap
 *  PUSH_Q_DEDUP    top-down, queue, the advance keeps duplicates and removes
 *                  them best-effort, without sorting (Table 3, variant 9): an
 *                  atomic-free block-mapped advance writes the depth and parent
 *                  of every target still unvisited in P_k and appends it to the
 *                  temporary list after dropping duplicates among the wave's
 *                  current candidates (an LDS hash of lane ids); a filter pass
 *                  then claims each entry as the atomic push does, so the next
 *                  frontier is exact.  Candidates beyond the list's
 *                  tmp_entries(n) are claimed in the advance itself
 * Every step emits the next frontier both as a queue and as a bitmap, so the
 * format of the next level is a free choice.
 */
#define BFS_V_PUSH_Q_THREAD 0
#define BFS_V_PUSH_Q_BLOCK 1
#define BFS_V_PUSH_Q_MERGE 2
#define BFS_V_PUSH_B_ATOMIC 3
#define BFS_V_PUSH_B_NOATOMIC 4
#define BFS_V_PUSH_Q_NOATOMIC 5
#define BFS_V_PULL_B 6
#define BFS_V_PULL_VIS 7         /* same depths, parents and scan lengths as BFS_V_PULL_B */
#define BFS_V_PUSH_P3 8
#define BFS_V_PUSH_Q_FILTER 9
#define BFS_V_PUSH_B_FILTER 10
#define BFS_V_PUSH_Q_DEDUP 11
#define BFS_NUM_VARIANTS 12
/* bfs_multi level_variant only: a split bottom-up level (options.hub_split). */
#define BFS_MS_SPLIT 200
/* Per-level choice modes. */
#define BFS_AUTO_HEURISTIC 100 /* Beamer direction-optimising rule (alpha 14, beta 24) */
#define BFS_AUTO_LEARNED 101   /* selector network on device; heuristic fallback */
#define BFS_SCHEDULE 102       /* options.schedule_host[k] at level k (last entry repeats) */

/* options.flags */
#define BFS_F_VALIDATE 1         /* check CSR/CSC structure before running (O(n+nnz)) */
#define BFS_F_STRICT_SELECTOR 2  /* learned mode without weights fails with BFS_ENOSEL */
#define BFS_F_LEVEL_STATS 4      /* fill the per-level arrays of bfs_stats */
#define BFS_F_DEVICE_LOOP 8      /* choose variants on the device and read the frontier
                                    size back only every few levels (fewer host syncs) */
#define BFS_F_LEVEL_TIMING 16    /* time each level's step with HIP events on the stream
                                    (fills level_ms; implies BFS_F_LEVEL_STATS) */
#define BFS_F_GRAPH_SUMS 32      /* options.graph_ld / graph_ld2 hold the graph-wide
                                    feature sums (from bfs_graph_sums): the call uses
                                    them instead of recomputing them over all vertices */
#define BFS_F_HUB_ORDER 64       /* bfs_multi: the graph is numbered by decreasing degree
                                    with ascending in-edge lists (bfs_reorder_degree), so
                                    the frontier bits its bottom-up steps read most often
                                    stay in cache and they skip the LDS frontier summary,
                                    and sparse bottom-up levels may be split at the heavy
                                    vertices (options.hub_split = 0) */
#define BFS_F_MAIN_TIMING 128    /* bfs_multi: time only each level's main kernel (fills
                                    level_ms_main, not level_ms; implies BFS_F_LEVEL_STATS):
                                    two HIP events per level instead of four */

/* ----------------------------------------------------------------- types */
typedef struct bfs_graph {
  int32_t n;               /* vertices, > 0 */
  int32_t nnz;             /* directed edges (CSR entries) */
  const int32_t *row_ptr;  /* device [n+1], out-edges of u in col_idx[row_ptr[u] .. row_ptr[u+1]) */
  const int32_t *col_idx;  /* device [nnz] */
  const int32_t *csc_ptr;  /* device [n+1] in-edges (transpose); may equal row_ptr for a
                              symmetric graph; NULL => pull variants unavailable */
  const int32_t *csc_idx;  /* device [nnz], ascending within each column for a
                              deterministic early exit */
} bfs_graph;

/* Tunable choices of bfs_multi's level steps (bfs_options.multi_config).  A
 * zero field takes the default in brackets.  No choice changes the depths,
 * only the time; bfs_multi_autotune picks them per graph.
 *   wide_ratio  non-split bottom-up levels run wide_vpt vertices per thread
 *               while the in-edges of the vertices still missing a lane
 *               exceed wide_ratio * n, narrow_vpt otherwise [8]
 *   split_vpt   vertices per thread on split bottom-up levels, 1, 2 or 4 [4]
 *   cap0        in-edges per pending vertex in the first round of a
 *               bottom-up level whose frontier holds more than a quarter of
 *               those in-edges (rounds grow 4x; sparser frontiers take every
 *               list in one round) [32]
 *   tile_alpha  bottom-up tiles: a 64-vertex chunk weighs at least
 *               tile_alpha per vertex, or its in-degree sum if larger, and a
 *               tile holds 256 * tile_alpha of weight, 16 .. 1024 [64]
 *   alpha       direction: bottom-up once the frontier's out-edges exceed
 *               1/alpha of the in-edges of the vertices still missing a lane
 *               (and n/8) [7]
 *   split_lout  with BFS_F_HUB_ORDER: a bottom-up level is split when the
 *               frontier holds at most a quarter of those in-edges and its
 *               light vertices' out-edges times split_lout are fewer [16]
 *   wide_vpt    see wide_ratio: 1, 2 or 4 [1]
 *   narrow_vpt  see wide_ratio: 1, 2 or 4 [4] */
typedef struct bfs_multi_config {
  int32_t wide_ratio;
  int32_t split_vpt;
  int32_t cap0;
  int32_t tile_alpha;
  int32_t alpha;
  int32_t split_lout;
  int32_t wide_vpt;
  int32_t narrow_vpt;
} bfs_multi_config;

typedef struct bfs_options {
  int32_t variant;               /* BFS_V_* or BFS_AUTO_* / BFS_SCHEDULE */
  int32_t flags;                 /* BFS_F_* */
  const int32_t *schedule_host;  /* BFS_SCHEDULE: variant per level */
  int32_t schedule_len;
  int32_t max_levels;            /* 0 => n + 1 */
  int32_t heuristic_push;        /* push variant used by the heuristic (-1 => default) */
  int32_t heuristic_pull;        /* pull variant used by the heuristic (-1 => default) */
  void *workspace;               /* device scratch, or NULL for a library-cached buffer */
  size_t workspace_bytes;
  int64_t graph_ld, graph_ld2;   /* with BFS_F_GRAPH_SUMS: the values bfs_graph_sums returned */
  const int32_t *vertex_map;     /* device [n] or NULL.  Set: the graph is a renumbered copy
                                    (bfs_reorder_degree, bfs_reorder_rcm) and vertex_map[v] is the new id of
                                    original vertex v (its new_of_old, a permutation of 0 .. n-1);
                                    sources, depths and parents are then in the original
                                    numbering.  bfs_multi, bfs_levels and bfs_parents; bfs_step_time
                                    returns BFS_ENOTSUP when it is set */
  int32_t hub_split;             /* bfs_multi only (the other calls ignore it): the split id T of
                                    split bottom-up levels.  On such a level the in-edges from
                                    vertices < T are pulled, reading each in-edge list only up to
                                    its first entry >= T, and the frontier vertices >= T push
                                    their out-edges first; together they cover every edge, so
                                    the depths do not depend on T.  0: T = the number of
                                    vertices of out-degree > 2048 when BFS_F_HUB_ORDER is set
                                    (they are vertices 0 .. T-1 there), used on the bottom-up
                                    levels where the frontier is sparse and its out-edges from
                                    vertices >= T are few; otherwise no split.  > 0: T =
                                    min(hub_split, n) on every bottom-up level.  < 0: never.
                                    A split needs every in-edge list in ascending order */
  const bfs_multi_config *multi_config; /* bfs_multi only: NULL => the configuration
                                    bfs_multi_autotune stored for this graph (same n, nnz,
                                    array addresses and BFS_F_HUB_ORDER), else the defaults */
} bfs_options;

typedef struct bfs_stats {
  int32_t num_levels;       /* 1 + largest depth */
  int32_t fell_back;        /* learned mode fell back to the heuristic at >= 1 level */
  int64_t reached;          /* vertices with depth >= 0 */
  int64_t component_edges;  /* sum of out-degrees of reached vertices (CSR entries) */
  float elapsed_ms;         /* device time from the first kernel to the last */
  int32_t host_syncs;       /* stream synchronisations the level loop made */
  /* Per-level arrays (host, caller-owned, level_capacity entries each; any may
   * be NULL); filled when BFS_F_LEVEL_STATS is set.  Entry k describes level k:
   * the variant that expanded F_k, |F_k|, out-edges of F_k, |U_k| and in-edges
   * of U_k, where U_k is the set unvisited after F_k was found. */
  int32_t level_capacity;
  int32_t *level_variant;
  int64_t *level_frontier;
  int64_t *level_frontier_edges;
  int64_t *level_unvisited;
  int64_t *level_unvisited_edges;
  int32_t *level_fallback;   /* learned mode: 1 where the heuristic decided */
  int64_t *level_frontier_ld;  /* sum over F_k of floor(log2(1 + outdeg)) */
  int64_t *level_frontier_ld2; /* sum over F_k of floor(log2(1 + outdeg))^2 */
  int64_t graph_ld, graph_ld2; /* the same two sums over all of V (learned mode or level stats) */
  int64_t *level_scanned;      /* edges examined by the step that expanded F_k */
  int64_t *level_next;         /* |F_{k+1}| found by that step */
  float *level_ms;             /* BFS_F_LEVEL_TIMING: device time of that step */
  /* bfs_multi only (untouched by the single-source calls): */
  float *level_ms_main;        /* BFS_F_LEVEL_TIMING: device time of the step's main kernel
                                  (bottom-up: the tile kernel; top-down: the light-source kernel) */
  int64_t *level_scanned_aux;  /* edges examined by the step's heavy-vertex kernel (part of level_scanned) */
  int64_t *level_hits_aux;     /* frontier words that kernel gathered (part of level_frontier_ld2) */
  int64_t *level_scanned_push; /* split level: edges examined by the push from vertices >= T
                                  (part of level_scanned); else 0 */
  int64_t *level_push_sources; /* split level: frontier vertices >= T that pushed; else 0 */
} bfs_stats;

/* Graph-wide sums over all vertices of floor(log2(1 + outdeg)) and of its
 * square: the two graph features of the learned per-level selector.  A caller
 * that searches one graph many times computes them once and passes them with
 * BFS_F_GRAPH_SUMS.  ld, ld2: host outputs.  Synchronises the stream. */
int bfs_graph_sums(const bfs_graph *g, int64_t *ld, int64_t *ld2, void *stream);

/* Renumbers the vertices by decreasing out-degree, ties by increasing id: a
 * preprocessing step (the paper renumbers every graph before timing, with
 * reverse Cuthill-McKee; Sec. "Experiment Setup").  New id i is the vertex
 * with the i-th largest out-degree, so the frontier words that bottom-up
 * steps read most often share few cache lines, and each ascending in-edge
 * list starts with its most connected in-neighbours (earlier exits).
 * Outputs, device, caller-allocated: out_row_ptr [n+1] and out_col_idx [nnz]
 * hold the renumbered CSR (edge (u, v) becomes (new u, new v)), rows
 * ascending; for a graph with its own CSC (csc_ptr set and != row_ptr)
 * out_csc_ptr [n+1] and out_csc_idx [nnz] hold the renumbered CSC (else they
 * are ignored: the result is symmetric too and its CSR serves as CSC);
 * new_of_old [n] and old_of_new [n] are the two directions of the map.
 * Validates the graph first (BFS_EGRAPH if malformed).  Allocates about
 * 16 * max(n, nnz) bytes of temporary device memory and synchronises the
 * stream. */
int bfs_reorder_degree(const bfs_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx,
                       int32_t *out_csc_ptr, int32_t *out_csc_idx, int32_t *new_of_old,
                       int32_t *old_of_new, void *stream);

/* The same outputs for reverse Cuthill-McKee, the renumbering the paper
 * applies to every graph (Sec. "Experiment Setup").  The paper does not
 * state its variant; this one works on the undirected structure (out-edges,
 * plus in-edges for a graph with its own CSC), deg(v) = the number of such
 * entries of v, and takes vertices in (deg, id) order: each component
 * starts at its remaining vertex first in that order, each visited vertex
 * appends its unvisited neighbours in that order (breadth first), and the
 * whole order is reversed.  The ordering pass runs on the host (one pass over
 * a copy of the graph); the rest, and the renumbering, on the GPU.
 * Validates the graph first; allocates as bfs_reorder_degree does, plus host
 * memory for a copy of the graph; synchronises the stream. */
int bfs_reorder_rcm(const bfs_graph *g, int32_t *out_row_ptr, int32_t *out_col_idx,
                    int32_t *out_csc_ptr, int32_t *out_csc_idx, int32_t *new_of_old,
                    int32_t *old_of_new, void *stream);

/* Workspace bytes for a graph of n vertices.  lanes = 1 for bfs_levels /
 * bfs_parents, 2..64 for bfs_multi (bit-packed lanes, u64 words per vertex). */
int bfs_workspace_size(int32_t n, int32_t lanes, size_t *bytes);

/* Single-source BFS depths.  levels: device [n] int32, written in full.
 * opt may be NULL (learned mode when weights are loaded, else heuristic).
 * st may be NULL. */
int bfs_levels(const bfs_graph *g, int32_t source, int32_t *levels,
               const bfs_options *opt, bfs_stats *st, void *stream);

/* As bfs_levels, and parents: device [n] int32.  parents[v] is some
 * in-neighbour of v at depth(v)-1 (the cascade's ANY reduction, Cascade 1,
 * Eq. advance: any one of the duplicate sources), so two runs may return
 * different but equally valid parents. */
int bfs_parents(const bfs_graph *g, int32_t source, int32_t *levels, int32_t *parents,
                const bfs_options *opt, bfs_stats *st, void *stream);

/* bfs_levels for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same search and
 * depths, with its scratch in a 32 MiB array the library holds on each GPU
 * for the life of the process instead of a workspace.  The call allocates no
 * device or host memory; it reads the loop state back into host stack memory
 * once per 16 levels.  Limits: n <= 724,928 (else BFS_EWORKSPACE);
 * options.workspace is ignored; BFS_F_LEVEL_STATS, BFS_F_LEVEL_TIMING and
 * BFS_F_DEVICE_LOOP return BFS_ENOTSUP (every level choice is made on the
 * device); st receives num_levels, reached, component_edges, fell_back,
 * host_syncs and elapsed_ms (host clock).  Every call on a GPU shares that
 * GPU's scratch and overwrites it (each call starts by resetting what it
 * reads): calls that overlap on one GPU, on any streams or threads, race. */
int bfs_levels_noalloc(const bfs_graph *g, int32_t source, int32_t *levels, const bfs_options *opt,
                       bfs_stats *st, void *stream);

/* Multi-source BFS over k sources (Cascade 1 started from several source nodes: one extra
 * lane rank on F and P).  Sources are processed in groups of up to 64 lanes;
 * lane l of vertex v lives in bit l of one u64 word, so a level is
 *     next[v] = (OR_{u in N_in(v)} front[u]) AND NOT vis[v]
 * on whole words.  sources_host: host [k]; levels: device [k][n] int32
 * (row i = depths from sources_host[i]).  st->component_edges sums over rows.
 * opt->variant: BFS_V_PUSH_Q_THREAD/BLOCK/MERGE select top-down, BFS_V_PULL_B
 * bottom-up, anything else the per-level heuristic.
 * With BFS_F_LEVEL_STATS (or BFS_F_LEVEL_TIMING) one per-level entry is
 * written per level of each 64-lane group, in order, and st->num_levels is
 * the number of entries: level_variant = BFS_V_PULL_B (bottom-up),
 * BFS_MS_SPLIT (bottom-up split at options.hub_split's T) or
 * BFS_V_PUSH_Q_THREAD (top-down); level_frontier / level_frontier_edges =
 * vertices in some lane's frontier and their out-edges; level_unvisited =
 * vertices missing some lane when the step started (bottom-up steps only,
 * else 0); level_unvisited_edges = in-edges of vertices missing some lane;
 * level_scanned = edges examined; level_next = (lane, vertex) pairs found;
 * level_frontier_ld = vertices with a lane found; level_frontier_ld2 = frontier
 * words gathered (one per examined in-edge whose source passed the frontier
 * bitmap probe, or per examined in-edge where a step gathers without it);
 * level_ms = step time.  Depths are written to `levels` once, by an output
 * pass after each group's last level (and by a flush pass every 255 levels).
 * With options.vertex_map (a graph from bfs_reorder_degree), sources_host
 * and the columns of `levels` are original vertex ids: the sources are
 * mapped on the device and the output pass reads each original vertex's
 * state at its new id. */
int bfs_multi(const bfs_graph *g, const int32_t *sources_host, int32_t k, int32_t *levels,
              const bfs_options *opt, bfs_stats *st, void *stream);

/* Tunes bfs_multi's configuration for one graph and source set: runs the
 * search (k sources, the same options otherwise) with candidate values of
 * each bfs_multi_config field in turn, keeping a candidate when its device
 * time (best of two runs) is at least 1% below the current choice's, starting
 * from options.multi_config or the defaults.
 * The result is returned in *best (and the time in *ms_best, may be NULL)
 * and stored for the graph, so later bfs_multi calls on it with
 * multi_config = NULL use it.  levels: device [k][n] scratch (holds the last
 * run's depths on return).  Takes some 25 configurations x 2 runs. */
int bfs_multi_autotune(const bfs_graph *g, const int32_t *sources_host, int32_t k, int32_t *levels,
                       const bfs_options *opt, bfs_multi_config *best, float *ms_best, void *stream);

/* ----------------------------------------------------------------- batch
 * Many independent graphs stored back to back (a disjoint union).  Instance b
 * owns global vertices [v_off[b], v_off[b+1]); row_ptr has total_n+1 GLOBAL
 * entry offsets; col_idx holds LOCAL vertex ids of the same instance.  All
 * instances are searched in one persistent launch (each level is Cascade 1's
 * step on that instance alone).  The instances are taken largest first from a
 * queue of tasks: an instance with n <= small_vertices is one task, searched
 * by one workgroup with its visited bitmap in LDS; a larger one is
 * G = min(ceil(n / team_vertices), max_team) tasks (1 when team_vertices is
 * 0), and the G workgroups that take them search it together, level by level,
 * behind a per-instance arrive counter.  A level goes bottom-up when the
 * in-edges it is expected to read (min(e_U, n_U (e_U + e_F) / e_F)) are fewer
 * than the frontier's out-edges (symmetric instances only). */
typedef struct bfs_graph_batch {
  int32_t num;               /* instances, > 0 */
  int32_t total_n;
  int32_t total_nnz;
  const int64_t *v_off_host; /* host [num+1] */
  const int64_t *e_off_host; /* host [num+1] */
  const int32_t *row_ptr;    /* device [total_n+1] */
  const int32_t *col_idx;    /* device [total_nnz] */
  int32_t symmetric;         /* 1: every instance is symmetric, so bottom-up steps may
                                use the CSR as in-edges; 0: top-down steps only */
} bfs_graph_batch;

typedef struct bfs_batch_config {
  int32_t block_threads;     /* 256, 512 or 1024 threads per workgroup */
  int32_t small_vertices;    /* instances with n <= this are searched by one workgroup with
                                the visited bitmap in LDS (and the bottom-up frontier bitmap
                                when both fit); at most 2^20 and what the device's LDS per
                                workgroup holds (BFS_EINVAL otherwise) */
  int32_t blocks_per_cu;     /* resident workgroups per compute unit (1..4; lowered to what
                                the kernel's registers and LDS allow) */
  int32_t team_vertices;     /* larger instances: vertices per team member (0: one member) */
  int32_t max_team;          /* most workgroups per team (1..16) */
  void *workspace;           /* device scratch of at least bfs_batch_workspace_size bytes,
                                or NULL for a buffer the library allocates and keeps */
  size_t workspace_bytes;
} bfs_batch_config;

/* Device scratch bytes bfs_batch needs for this batch and config (cfg NULL:
 * the config bfs_batch would use).  Host-only; sources_host as for bfs_batch. */
int bfs_batch_workspace_size(const bfs_graph_batch *b, const int32_t *sources_host,
                             const bfs_batch_config *cfg, size_t *bytes);

/* levels: device [total_n] int32, per instance in local depth terms.
 * sources_host: host [num] local ids.  cfg NULL => defaults (or the last
 * autotuned config for a batch of the same signature) with a library-kept
 * workspace.  Returns BFS_EHIP if a team's wait for its members ran out (2 s;
 * only when other work on the device keeps part of the grid from running). */
int bfs_batch(const bfs_graph_batch *b, const int32_t *sources_host, int32_t *levels,
              const bfs_batch_config *cfg, bfs_stats *st, void *stream);

/* Times candidate configs (threads per workgroup, small-instance threshold,
 * team_vertices, max_team) on this batch and returns the fastest in *best
 * (and caches it under the batch's size signature).  best->workspace /
 * workspace_bytes, if set on entry, serve every candidate (candidates that
 * need more are skipped).  levels is device scratch of total_n ints.
 * ms_best may be NULL. */
int bfs_batch_autotune(const bfs_graph_batch *b, const int32_t *sources_host, int32_t *levels,
                       bfs_batch_config *best, float *ms_best, void *stream);

/* -------------------------------------------------------------- selector
 * Per-level variant selector: 12 features -> 64 -> 64 -> 4 (ReLU), weights
 * used in bfloat16 (round to nearest even), layer inputs rounded to bfloat16,
 * fp32 accumulation starting from the bias in ascending input order.
 * Parameter layout (5,252 fp32): W1[64][12], b1[64], W2[64][64], b2[64],
 * W3[4][64], b3[4]; weights are [out][in] row-major.
 * Features of level k, with ld(v) = floor(log2(1 + outdeg(v))) (exact
 * integer sums; computed in fp64, then rounded to fp32):
 *   0 log2(1+|F|)  1 log2(1+eF)  2 log2(1+|U|)  3 log2(1+eU)
 *   4 |F|/n  5 eF/nnz  6 |U|/n  7 mean of ld over F  8 variance of ld over F
 *   9 mean of ld over V  10 variance of ld over V  11 log2(1+k)
 * normalised as (x - mean) / std in fp32.  The selector falls back to the
 * heuristic at a level when the top softmax probability is below
 * min_confidence or a raw feature lies outside [feat_min, feat_max]. */
#define BFS_MLP_NPARAM 5252
#define BFS_MLP_NFEAT 12
#define BFS_MLP_NCLASS 4
int bfs_selector_set(const float *params_host, const float *feat_mean_host,
                     const float *feat_std_host, const float *feat_min_host,
                     const float *feat_max_host, float min_confidence,
                     const int32_t *class_variant_host /* [4] BFS_V_* */);
/* Loads selector weights from a file (the persisted form of the trained
 * network, so a C caller can use BFS_AUTO_LEARNED without Python).  Layout,
 * little-endian, 21,244 bytes:
 *   bytes 0..7     magic "BFSSEL01"
 *   uint32 x 4     version (1), parameter count (5,252), features (12), classes (4)
 *   float32 x 5252 parameters in the layout above
 *   float32 x 12   feature mean      float32 x 12  feature std (> 0)
 *   float32 x 12   training minimum  float32 x 12  training maximum
 *   float32        min_confidence
 *   int32 x 4      BFS_V_* variant of each class
 * The file is read and checked in full before anything is loaded: a missing,
 * short or long file, a wrong header, a non-finite value, a std <= 0 or a
 * class outside the variant range returns BFS_EFILE and leaves the loaded
 * selector (if any) unchanged.  Otherwise as bfs_selector_set (which
 * allocates the device copy of the weights on first use per device). */
int bfs_selector_load(const char *path);
int bfs_selector_clear(void);
int bfs_selector_loaded(void);

/* Training kernels (device pointers; used by the selector's trainer and by
 * the gradient checks).  x: [batch][12] normalised features. */
int bfs_mlp_forward(const float *params, const float *x, int32_t batch, float *logits,
                    void *stream);
/* Mean softmax cross-entropy loss (device scalar) and its gradient w.r.t. the
 * fp32 master parameters (straight-through through every bf16 rounding). */
int bfs_mlp_loss_grad(const float *params, const float *x, const int32_t *labels,
                      int32_t batch, float *grad, float *loss, void *stream);
/* One Adam step (Kingma & Ba, bias-corrected) on params in place. */
int bfs_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream);
/* Argmax class (ties to the lowest index) and top softmax probability. */
int bfs_mlp_predict(const float *params, const float *x, int32_t batch, int32_t *cls,
                    float *conf, void *stream);
/* Raw (unnormalised) features of every level recorded in st (filled by a
 * bfs_levels/bfs_parents call with BFS_F_LEVEL_STATS and all per-level
 * arrays), computed by the same code the device selector runs.
 * feats_host: host [st->num_levels][12]. */
int bfs_level_features(const bfs_stats *st, int32_t n, int32_t nnz, float *feats_host);

/* ------------------------------------------------------- per-level timing
 * Restores the exact state of level k from the depths of a finished search
 * (F_k = {depth = k}, P_k = {0 <= depth <= k}), runs one step of `variant`
 * `reps` times from that state and returns the median device time in ms.
 * depths: device [n] (read only); scratch_levels: device [n]. */
int bfs_step_time(const bfs_graph *g, const int32_t *depths, int32_t k, int32_t variant,
                  int32_t reps, int32_t *scratch_levels, const bfs_options *opt,
                  float *ms_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BFS_EEDS_H */
