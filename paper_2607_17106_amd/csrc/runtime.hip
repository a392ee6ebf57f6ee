// Host runtime of the single-source BFS: workspace layout, the per-level
// loop (Cascade 1 iterated until the frontier is empty), per-level variant
// choice, statistics and the C ABI entry points bfs_levels / bfs_parents.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "selector.hpp"
#include "persist.hpp"

namespace bfs {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return BFS_EHIP;
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static inline int words_of(int n) { return (n + 63) / 64; }

constexpr int GSUM_WORDS = 1280;  // graph sums, selector state, flag, 64 partial lines

static size_t single_core_bytes(int n) {
  const size_t W = (size_t)words_of(n);
  size_t b = 0;
  b += align256(W * 8);                              // vis
  b += 3 * align256(W * 8);                          // fb[3]
  b += 2 * align256(queue_entries(n) * 4);           // q[2]
  b += align256(((size_t)n + 1) * 4);                // scan
  b += align256(((size_t)n / SCAN_CHUNK + 2) * 4);   // bsum
  b += align256((size_t)n * 4);                      // hubs
  b += align256(RING * sizeof(RingSlot));            // ring
  b += align256(LOGCAP * sizeof(LevelLog));          // log
  b += align256(sizeof(LoopCtl));                    // ctl
  b += align256(sizeof(GridBar));                    // bar
  b += align256(LOGCAP * sizeof(int));               // sched
  b += align256(GSUM_WORDS * 8);                     // gsum
  b += align256(W * 8);                              // vis_prev
  b += align256(sizeof(int));                        // p3_level
  b += 2 * align256((size_t)tmp_entries(n) * 4);     // tmp_v, tmp_u
  return b;
}

// After the layout carve_single cuts: with options.vertex_map, the depths and
// parents in the graph's numbering and the inverse map (n ints each).
size_t workspace_bytes_single(int n) { return single_core_bytes(n) + 3 * align256((size_t)n * 4); }

struct MapBufs {
  int *lv, *par, *inv;
};
static MapBufs map_bufs(void *base, int n) {
  char *p = static_cast<char *>(base) + single_core_bytes(n);
  const size_t b = align256((size_t)n * 4);
  return MapBufs{reinterpret_cast<int *>(p), reinterpret_cast<int *>(p + b), reinterpret_cast<int *>(p + 2 * b)};
}

// inv[map[v]] = v (map: a permutation of 0 .. n-1).
__global__ __launch_bounds__(BLOCK) void k_invert_map(const int *map, int *inv, int n) {
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < n; v += gridDim.x * BLOCK) inv[map[v]] = v;
}

// Depths (and parents) of the renumbered graph's search at the original ids:
// lv[v] = lv_new[map[v]], par[v] = inv[par_new[map[v]]] (or -1).
__global__ __launch_bounds__(BLOCK) void k_unmap(const int *map, const int *inv, const int *lv_new,
                                                 const int *par_new, int *lv, int *par, int n) {
  for (int v = blockIdx.x * BLOCK + threadIdx.x; v < n; v += gridDim.x * BLOCK) {
    const int m = map[v];
    lv[v] = lv_new[m];
    if (par) {
      const int p = par_new[m];
      par[v] = p >= 0 ? inv[p] : -1;
    }
  }
}

Workspace carve_single(void *base, int n) {
  Workspace w;
  const size_t W = (size_t)words_of(n);
  char *p = (char *)base;
  auto take = [&](size_t bytes) { char *r = p; p += align256(bytes); return (void *)r; };
  w.vis = (u64 *)take(W * 8);
  for (int i = 0; i < 3; ++i) w.fb[i] = (u64 *)take(W * 8);
  for (int i = 0; i < 2; ++i) w.q[i] = (int *)take(queue_entries(n) * 4);
  w.scan = (int *)take(((size_t)n + 1) * 4);
  w.bsum = (int *)take(((size_t)n / SCAN_CHUNK + 2) * 4);
  w.hubs = (int *)take((size_t)n * 4);
  w.ring = (RingSlot *)take(RING * sizeof(RingSlot));
  w.log = (LevelLog *)take(LOGCAP * sizeof(LevelLog));
  w.ctl = (LoopCtl *)take(sizeof(LoopCtl));
  w.bar = take(sizeof(GridBar));
  w.sched = (int *)take(LOGCAP * sizeof(int));
  w.gsum = (u64 *)take(GSUM_WORDS * 8);
  w.vis_prev = (u64 *)take(W * 8);
  w.p3_level = (int *)take(sizeof(int));
  w.tmp_v = (int *)take((size_t)tmp_entries(n) * 4);
  w.tmp_u = (int *)take((size_t)tmp_entries(n) * 4);
  w.W = (int)W;
  w.qcap = queue_cap(n);
  return w;
}

// ------------------------------------------------- per-thread host context
HostCtx::HostCtx() {
  // coherent (fine-grained): a kernel's stores reach the host while it still
  // runs, so the host can poll the sequence word a level's last kernel posts
  if (hipHostMalloc((void **)&pinned, 64 * sizeof(LevelCtr), hipHostMallocCoherent) != hipSuccess) return;
  pinned_u64 = reinterpret_cast<u64 *>(pinned + 32);
  // ev[0] / ev[1] bracket a whole call (the host waits on ev[1]); the others
  // only time steps, so they skip the system-scope cache writeback and
  // invalidate a default event performs when it is recorded
  for (int i = 0; i < 4; ++i)
    if (hipEventCreateWithFlags(&ev[i], i < 2 ? hipEventDefault : hipEventDisableSystemFence) != hipSuccess) return;
  for (int i = 0; i < 64; ++i)
    if (hipEventCreateWithFlags(&lev_ev[i], hipEventDisableSystemFence) != hipSuccess) return;
  ok = true;
}

int wait_posted(const volatile u64 *flag, u64 seq, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned spin = 0; *flag != seq; ++spin) {
    if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
      BFS_HIP(hipStreamSynchronize(s));
      if (*flag != seq) {
        set_error("level totals were not posted by the device");
        return BFS_EHIP;
      }
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return BFS_OK;
}

HostCtx &host_ctx() {
  static thread_local HostCtx c;
  return c;
}

// Library-cached workspace for callers that pass none (one per device).
static std::mutex g_ws_mu;
static void *g_ws_ptr[64] = {nullptr};
static size_t g_ws_len[64] = {0};

int cached_workspace(size_t bytes, void **out) {
  int dev = 0;
  BFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return BFS_EINVAL;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (g_ws_len[dev] < bytes) {
    if (g_ws_ptr[dev]) BFS_HIP(hipFree(g_ws_ptr[dev]));
    g_ws_ptr[dev] = nullptr;
    g_ws_len[dev] = 0;
    BFS_HIP(hipMalloc(&g_ws_ptr[dev], bytes));
    g_ws_len[dev] = bytes;
  }
  *out = g_ws_ptr[dev];
  return BFS_OK;
}

int check_graph(const bfs_graph *g) {
  if (!g || g->n <= 0 || g->nnz < 0 || !g->row_ptr || (!g->col_idx && g->nnz > 0)) {
    set_error("invalid graph (null pointer, n <= 0 or nnz < 0)");
    return BFS_EINVAL;
  }
  if ((g->csc_ptr && !g->csc_idx && g->nnz > 0) || (!g->csc_ptr && g->csc_idx)) {
    set_error("csc_ptr and csc_idx must both be given or both be NULL");
    return BFS_EINVAL;
  }
  return BFS_OK;
}

int validate_graph(const bfs_graph *g, u64 *flag_dev, hipStream_t s) {
  HostCtx &hc = host_ctx();
  BFS_HIP(hipMemsetAsync(flag_dev, 0, 8, s));
  BFS_HIP(launch_validate(g->n, g->nnz, g->row_ptr, g->col_idx, flag_dev, s));
  if (g->csc_ptr && g->csc_ptr != g->row_ptr)
    BFS_HIP(launch_validate(g->n, g->nnz, g->csc_ptr, g->csc_idx, flag_dev, s));
  BFS_HIP(hipMemcpyAsync(hc.pinned_u64, flag_dev, 8, hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  if (*hc.pinned_u64) {
    set_error("malformed graph: %s%s", (*hc.pinned_u64 & 1) ? "bad offsets " : "",
              (*hc.pinned_u64 & 2) ? "column id out of range" : "");
    return BFS_EGRAPH;
  }
  return BFS_OK;
}

// ------------------------------------------------------ direction rule
// Beamer, Asanovic, Patterson (SC'12): top-down -> bottom-up when
// m_f > m_u / alpha; bottom-up -> top-down when n_f < n / beta and the
// frontier shrank.  alpha = 14, beta = 24.
void HeuristicState::step(long long n, long long nF, long long eF, long long eU) {
  if (dir == 0) {
    if (eF * kAlpha > eU) dir = 1;
  } else {
    bool shrinking = prev_nf >= 0 && nF < prev_nf;
    if (nF * kBeta < n && shrinking) dir = 0;
  }
  prev_nf = nF;
}

static bool is_pull(int v) { return v == BFS_V_PULL_B || v == BFS_V_PULL_VIS; }

// Device wall-clock rate in kHz (ticks per millisecond).
static double wall_khz() {
  static double khz = 0.0;
  if (khz == 0.0) {
    int dev = 0, r = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&r, hipDeviceAttributeWallClockRate, dev) == hipSuccess && r > 0)
      khz = (double)r;
    else
      khz = 100000.0;
  }
  return khz;
}

hipError_t launch_log_f0(RingSlot *slot0, LevelLog *log, LoopCtl *ctl, hipStream_t s);
static hipError_t launch_finish_f0(const Workspace &w, hipStream_t s) {
  return launch_log_f0(w.ring, w.log, w.ctl, s);
}

// Graph-wide sums of floor(log2(1 + outdeg)) and of its square (selector
// features): computed over all vertices and read back (one stream sync).
static int graph_ld_sums(const bfs_graph *g, const Workspace &w, hipStream_t s, u64 *ld, u64 *ld2) {
  HostCtx &hc = host_ctx();
  BFS_HIP(launch_graph_ld(g->n, g->row_ptr, w.gsum, s));
  BFS_HIP(hipMemcpyAsync(hc.pinned_u64, w.gsum, 16, hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  *ld = hc.pinned_u64[0];
  *ld2 = hc.pinned_u64[1];
  return BFS_OK;
}

// Degree above which the block-mapped and bitmap pushes defer a frontier
// vertex to the grid-wide hub pass.  Those pushes give each workgroup up to
// BLOCK frontier vertices, so with a small frontier the lists of a whole level
// would sit on one or two workgroups: the threshold then drops and nearly every
// list is spread over the grid.
static int hub_threshold(long long frontier) { return frontier < 64LL * BLOCK ? 64 : DEFAULT_HUB; }

static StepArgs level_args(const bfs_graph *g, const Workspace &w, int *levels, int *parents, int k, int hub) {
  StepArgs a;
  a.gate = -1;
  a.n = g->n;
  a.W = w.W;
  a.k = k;
  a.hub = hub;
  a.qcap = w.qcap;
  a.rp = g->row_ptr;
  a.ci = g->col_idx;
  a.cp = g->csc_ptr;
  a.cx = g->csc_idx;
  a.levels = levels;
  a.parents = parents;
  a.vis = w.vis;
  a.vis_prev = w.vis_prev;
  a.p3_level = w.p3_level;
  a.tmp_v = w.tmp_v;
  a.tmp_u = w.tmp_u;
  a.tmpcap = tmp_entries(g->n);
  a.nnz = g->nnz;
  a.fb_cur = w.fb[k % 3];
  a.fb_next = w.fb[(k + 1) % 3];
  a.fb_dead = w.fb[(k + 2) % 3];
  a.q_cur = w.q[k % 2];
  a.q_next = w.q[(k + 1) % 2];
  a.c_cur = &w.ring[k % RING].tot;
  a.seg_cur = w.ring[k % RING].seg;
  a.sh_next = w.ring[(k + 1) % RING].sh;
  a.sh_zero = w.ring[(k + 2) % RING].sh;
  a.scan = w.scan;
  a.bsum = w.bsum;
  a.hubs = w.hubs;
  return a;
}

static int run_single(const bfs_graph *g, int src, int *levels, int *parents, const bfs_options *opt_in,
                      bfs_stats *st, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (src < 0 || src >= g->n) {
    set_error("source %d out of range [0, %d)", src, g->n);
    return BFS_EINVAL;
  }
  bfs_options dflt;
  memset(&dflt, 0, sizeof(dflt));
  dflt.variant = selector_loaded() ? BFS_AUTO_LEARNED : BFS_AUTO_HEURISTIC;
  dflt.heuristic_push = -1;
  dflt.heuristic_pull = -1;
  const bfs_options *opt = opt_in ? opt_in : &dflt;
  int mode = opt->variant;
  const bool have_csc = g->csc_ptr != nullptr;
  if (mode >= 0 && mode < BFS_NUM_VARIANTS) {
    if (is_pull(mode) && !have_csc) {
      set_error("pull variant needs CSC arrays");
      return BFS_ENOTSUP;
    }
  } else if (mode == BFS_SCHEDULE) {
    if (!opt->schedule_host || opt->schedule_len <= 0) {
      set_error("BFS_SCHEDULE needs schedule_host and schedule_len > 0");
      return BFS_EINVAL;
    }
    for (int i = 0; i < opt->schedule_len; ++i) {
      int v = opt->schedule_host[i];
      if (v < 0 || v >= BFS_NUM_VARIANTS) {
        set_error("schedule entry %d is not a variant id", i);
        return BFS_EINVAL;
      }
      if (is_pull(v) && !have_csc) {
        set_error("schedule uses a pull variant but no CSC arrays were given");
        return BFS_ENOTSUP;
      }
    }
  } else if (mode != BFS_AUTO_HEURISTIC && mode != BFS_AUTO_LEARNED) {
    set_error("unknown variant/mode %d", mode);
    return BFS_EINVAL;
  }
  bool learned = mode == BFS_AUTO_LEARNED;
  int fell_back_all = 0;
  if (learned && !selector_loaded()) {
    if (opt->flags & BFS_F_STRICT_SELECTOR) {
      set_error("learned mode requested but no selector weights are loaded");
      return BFS_ENOSEL;
    }
    learned = false;
    mode = BFS_AUTO_HEURISTIC;
    fell_back_all = 1;
  }
  const bool device_decides = (mode == BFS_AUTO_HEURISTIC || mode == BFS_AUTO_LEARNED);
  int push_v = (opt->heuristic_push >= 0 && opt->heuristic_push < BFS_NUM_VARIANTS && !is_pull(opt->heuristic_push))
                   ? opt->heuristic_push : BFS_V_PUSH_Q_BLOCK;
  int pull_v = have_csc ? BFS_V_PULL_B : push_v;

  HostCtx &hc = host_ctx();
  if (!hc.ok) {
    set_error("pinned host buffer or event creation failed");
    return BFS_EHIP;
  }
  const size_t need = workspace_bytes_single(g->n);
  void *wsp = opt->workspace;
  if (wsp) {
    if (opt->workspace_bytes < need) {
      set_error("workspace has %zu bytes, needs %zu", opt->workspace_bytes, need);
      return BFS_EWORKSPACE;
    }
  } else {
    rc = cached_workspace(need, &wsp);
    if (rc) return rc;
  }
  Workspace w = carve_single(wsp, g->n);
  if (opt->flags & BFS_F_VALIDATE) {
    rc = validate_graph(g, w.gsum + 8, s);
    if (rc) return rc;
  }
  // vertex_map (a renumbered graph): the search runs in the graph's numbering
  // from the source's new id, into workspace buffers, and a last pass writes
  // depths (and parents) at the original ids
  const int *vmap = opt->vertex_map;
  int *levels_out = levels, *parents_out = parents;
  const MapBufs mb = map_bufs(wsp, g->n);
  if (vmap) {
    BFS_HIP(hipMemcpyAsync(hc.pinned_u64 + 24, vmap + src, sizeof(int), hipMemcpyDeviceToHost, s));
    BFS_HIP(hipStreamSynchronize(s));
    src = reinterpret_cast<const int *>(hc.pinned_u64 + 24)[0];
    if (src < 0 || src >= g->n) {
      set_error("vertex_map maps the source to %d, outside [0, %d)", src, g->n);
      return BFS_EINVAL;
    }
    levels = mb.lv;
    parents = parents ? mb.par : nullptr;
  }
  const long long maxlev = opt->max_levels > 0 ? opt->max_levels : (long long)g->n + 1;
  const bool want_levels =
      st && (opt->flags & (BFS_F_LEVEL_STATS | BFS_F_LEVEL_TIMING)) && st->level_capacity > 0;
  const bool timing = want_levels && (opt->flags & BFS_F_LEVEL_TIMING);
  const bool device_loop = (opt->flags & BFS_F_DEVICE_LOOP) != 0;
  // variants a device-decided level may pick
  std::vector<int> cands;
  if (device_decides) {
    cands.push_back(push_v);
    if (pull_v != push_v) cands.push_back(pull_v);
    if (learned) {
      SelDevice probe = selector_device(w, push_v, pull_v);
      for (int c = 0; c < NC; ++c) {
        int v = probe.cls[c];
        if (is_pull(v) && !have_csc) continue;
        if (std::find(cands.begin(), cands.end(), v) == cands.end()) cands.push_back(v);
      }
    }
  }
  auto fixed_variant = [&](int k) -> int {
    if (mode >= 0 && mode < BFS_NUM_VARIANTS) return mode;
    return opt->schedule_host[std::min(k, opt->schedule_len - 1)];
  };

  const bool host_loop = !device_loop;  // the level totals reach the host by posts, level by level
  BFS_HIP(hipEventRecord(hc.ev[0], s));
  if (!host_loop) BFS_HIP(hipMemsetAsync(w.ctl, 0, sizeof(LoopCtl), s));  // the host loop's first launch sets it
  const bool graph_sums = learned || want_levels;
  u64 gld = 0, gld2 = 0;
  if (graph_sums) {
    if (opt->flags & BFS_F_GRAPH_SUMS) {
      gld = (u64)opt->graph_ld;
      gld2 = (u64)opt->graph_ld2;
    } else {
      rc = graph_ld_sums(g, w, s, &gld, &gld2);
      if (rc) return rc;
    }
  }
  StepArgs a = level_args(g, w, levels, parents, 0, DEFAULT_HUB);
  SelDevice seldev = selector_device(w, push_v, pull_v);
  seldev.gld = gld;
  seldev.gld2 = gld2;
  bool persistent = device_loop;
  if (persistent) {
    PersistArgs P;
    P.base = a;
    for (int i = 0; i < 3; ++i) P.fb[i] = w.fb[i];
    for (int i = 0; i < 2; ++i) P.q[i] = w.q[i];
    P.ring = w.ring;
    P.log = w.log;
    P.ctl = w.ctl;
    P.gsum = w.gsum;
    P.bar = reinterpret_cast<GridBar *>(w.bar);
    P.decide = device_decides ? 1 : 0;
    P.use_net = learned ? 1 : 0;
    P.maxlev = (int)std::min<long long>(maxlev, (long long)INT32_MAX);
    P.src = src;
    P.nnz = g->nnz;
    P.push_v = push_v;
    P.sd = seldev;
    P.sched = w.sched;
    P.sched_len = 1;
    if (!device_decides) {
      std::vector<int> sv;
      if (mode == BFS_SCHEDULE) {
        sv.assign(opt->schedule_host, opt->schedule_host + std::min(opt->schedule_len, LOGCAP));
      } else {
        sv.push_back(mode);
      }
      P.sched_len = (int)sv.size();
      BFS_HIP(hipMemcpyAsync(w.sched, sv.data(), sv.size() * sizeof(int), hipMemcpyHostToDevice, s));
    }
    BFS_HIP(hipMemsetAsync(w.bar, 0, sizeof(GridBar), s));
    hipError_t le = launch_persistent(P, s);
    if (le != hipSuccess) {
      (void)hipGetLastError();  // fall back to the launch-ahead loop below
      persistent = false;
    }
  }
  u64 start_seq = 0;
  if (!persistent && !device_loop) {
    // host loop: level 0 set up, chosen and posted by one launch after the reset
    BFS_HIP(launch_reset(a, src, w.ring, s, false));
    start_seq = ++hc.seq;
    BFS_HIP(launch_start_select(g->row_ptr, g->csc_ptr, src, w.ring, w.log, w.ctl, seldev, g->n, g->nnz,
                                device_decides, learned, hc.pinned, hc.pinned_u64 + 255, start_seq, s));
  } else if (!persistent) {
    BFS_HIP(launch_reset(a, src, w.ring, s));
    BFS_HIP(launch_finish_f0(w, s));
    if (device_decides) BFS_HIP(launch_select(seldev, w.ring, 0, g->n, g->nnz, s, true, learned, w.log));
  }

  int syncs = 0;
  int k = 0;
  std::vector<int> host_variant;  // variants the host chose (fixed / schedule modes)
  std::vector<float> level_ms;
  // host loop: the loop control's totals and the fallback flags, gathered
  // from the posts (the same sums the device keeps in LoopCtl)
  long long h_levels = 0, h_reached = 0, h_comp = 0;
  int h_fb = 0;
  if (!device_loop) {
    rc = wait_posted(hc.pinned_u64 + 255, start_seq, s);
    if (rc) return rc;
    ++syncs;
    long long cnt = hc.pinned[0].count;
    long long eF = (long long)hc.pinned[0].edges;
    int dec = hc.pinned[0].decision;
    h_levels = 1;
    h_reached = cnt;
    h_comp = eF;
    h_fb = hc.pinned[0].fallback;
    for (;;) {
      int v = device_decides ? dec : fixed_variant(k);
      if (v < 0 || v >= BFS_NUM_VARIANTS || (is_pull(v) && !have_csc)) v = push_v;
      host_variant.push_back(v);
      a = level_args(g, w, levels, parents, k, hub_threshold(cnt));
      a.gate = -1;
      if (timing) BFS_HIP(hipEventRecord(hc.ev[2], s));
      BFS_HIP(launch_step(v, a, (int)cnt, eF, s));
      if (timing) BFS_HIP(hipEventRecord(hc.ev[3], s));
      {
        u64 *seq_word = hc.pinned_u64 + 255;
        const u64 seq = ++hc.seq;
        BFS_HIP(launch_finish_select(&w.ring[(k + 1) % RING], w.qcap, k + 1, w.log, w.ctl, seldev, w.ring, g->n,
                                     g->nnz, device_decides, learned, hc.pinned, seq_word, seq, s));
        rc = wait_posted(seq_word, seq, s);
        if (rc) return rc;
      }
      ++syncs;
      if (timing) {
        float ms = 0.f;
        // the post can be seen before the runtime has marked the event done
        BFS_HIP(hipEventSynchronize(hc.ev[3]));
        BFS_HIP(hipEventElapsedTime(&ms, hc.ev[2], hc.ev[3]));
        level_ms.push_back(ms);
      }
      const LevelCtr c = hc.pinned[0];
      if (c.count == 0) break;
      cnt = c.count;
      eF = (long long)c.edges;
      dec = c.decision;
      h_levels = k + 2;
      h_reached += cnt;
      h_comp += eF;
      h_fb |= c.fallback;
      ++k;
      if (k >= maxlev) {
        set_error("level loop reached max_levels = %lld", maxlev);
        return BFS_ELEVELCAP;
      }
    }
  } else if (!persistent) {
    // Enqueue BATCH levels ahead; every step kernel checks the device-side
    // decision (gate) and the frontier size, so levels past the end are
    // no-ops.  The host reads the loop control once per batch.
    constexpr int BATCH = 16;
    hipEvent_t *evs = hc.lev_ev;
    bool done = false;
    while (!done) {
      const int k0 = k;
      for (int i = 0; i < BATCH; ++i, ++k) {
        a = level_args(g, w, levels, parents, k, DEFAULT_HUB);
        if (timing) BFS_HIP(hipEventRecord(evs[2 * i], s));
        if (device_decides) {
          for (int v : cands) {
            a.gate = v;
            BFS_HIP(launch_step(v, a, -1, -1, s));
          }
        } else {
          a.gate = -2;
          int v = fixed_variant(k);
          host_variant.push_back(v);
          BFS_HIP(launch_step(v, a, -1, -1, s));
        }
        if (timing) BFS_HIP(hipEventRecord(evs[2 * i + 1], s));
        BFS_HIP(launch_finish_select(&w.ring[(k + 1) % RING], w.qcap, k + 1, w.log, w.ctl, seldev, w.ring, g->n,
                                     g->nnz, device_decides, learned, nullptr, nullptr, 0, s));
      }
      BFS_HIP(hipMemcpyAsync(hc.pinned_u64, w.ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, s));
      BFS_HIP(hipStreamSynchronize(s));
      ++syncs;
      const LoopCtl *c = reinterpret_cast<const LoopCtl *>(hc.pinned_u64);
      done = c->done != 0;
      if (timing) {
        const int last = done ? std::min((int)c->levels, k) : k;
        for (int i = 0; i < BATCH && k0 + i < last; ++i) {
          float ms = 0.f;
          BFS_HIP(hipEventElapsedTime(&ms, evs[2 * i], evs[2 * i + 1]));
          level_ms.push_back(ms);
        }
      }
      if (!done && k >= maxlev) {
        set_error("level loop reached max_levels = %lld", maxlev);
        return BFS_ELEVELCAP;
      }
    }
  }
  if (vmap) {
    const int grid = std::min(4096, (g->n + BLOCK - 1) / BLOCK);
    if (parents_out) hipLaunchKernelGGL(k_invert_map, dim3(grid), dim3(BLOCK), 0, s, vmap, mb.inv, g->n);
    hipLaunchKernelGGL(k_unmap, dim3(grid), dim3(BLOCK), 0, s, vmap, (const int *)mb.inv, (const int *)mb.lv,
                       (const int *)(parents_out ? mb.par : nullptr), levels_out, parents_out, g->n);
    BFS_HIP(hipGetLastError());
  }
  BFS_HIP(hipEventRecord(hc.ev[1], s));
  LoopCtl ctl;
  if (host_loop) {  // every total is on the host already: wait for the last kernel only
    BFS_HIP(hipEventSynchronize(hc.ev[1]));
    memset(&ctl, 0, sizeof(ctl));
    ctl.done = 1;
    ctl.levels = (u64)h_levels;
    ctl.reached = (u64)h_reached;
    ctl.comp_edges = (u64)h_comp;
  } else {
    BFS_HIP(hipMemcpyAsync(hc.pinned_u64, w.ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, s));
    BFS_HIP(hipEventSynchronize(hc.ev[1]));
    BFS_HIP(hipStreamSynchronize(s));
    memcpy(&ctl, hc.pinned_u64, sizeof(ctl));
  }
  if (persistent) {
    BFS_HIP(hipMemcpy(hc.pinned_u64 + 16, &reinterpret_cast<GridBar *>(w.bar)->err.v, 4, hipMemcpyDeviceToHost));
    if (reinterpret_cast<u32 *>(hc.pinned_u64 + 16)[0] != 0u) {
      set_error("persistent search: a grid barrier timed out");
      return BFS_EHIP;
    }
    if (ctl.pad[0] == 2) {
      set_error("level loop reached max_levels = %lld", maxlev);
      return BFS_ELEVELCAP;
    }
    syncs = 1;
    if (mode >= 0 && mode < BFS_NUM_VARIANTS) host_variant.assign((size_t)ctl.levels + 1, mode);
    if (mode == BFS_SCHEDULE)
      for (int i = 0; i <= (int)ctl.levels; ++i)
        host_variant.push_back(opt->schedule_host[std::min(i, opt->schedule_len - 1)]);
  }
  const int nlev = (int)ctl.levels;
  if (nlev > maxlev) {
    set_error("level loop reached max_levels = %lld", maxlev);
    return BFS_ELEVELCAP;
  }
  if (!st) return BFS_OK;
  float ms = 0.f;
  BFS_HIP(hipEventElapsedTime(&ms, hc.ev[0], hc.ev[1]));
  st->num_levels = nlev;
  st->reached = (int64_t)ctl.reached;
  st->component_edges = (int64_t)ctl.comp_edges;
  st->elapsed_ms = ms;
  st->host_syncs = syncs;
  st->fell_back = fell_back_all;
  if (graph_sums) {
    st->graph_ld = (int64_t)gld;
    st->graph_ld2 = (int64_t)gld2;
  }
  // per-level statistics from the device log (entry k+1 also carries the
  // scan length of the step that expanded F_k)
  if (host_loop) st->fell_back |= h_fb;
  if (host_loop && !want_levels) return BFS_OK;
  const int L = std::min(nlev + 1, LOGCAP);
  std::vector<LevelLog> lg(L);
  BFS_HIP(hipMemcpy(lg.data(), w.log, L * sizeof(LevelLog), hipMemcpyDeviceToHost));
  int any_fb = 0;
  for (int k2 = 0; k2 < std::min(nlev, L); ++k2) any_fb |= lg[k2].fallback;
  st->fell_back |= any_fb;
  if (!want_levels) return BFS_OK;
  long long nU = g->n, eU = g->nnz;
  const int cap = std::min(st->level_capacity, L - 1 >= 0 ? L - 1 : 0);
  for (int k2 = 0; k2 < std::min(nlev, cap); ++k2) {
    const LevelLog &e = lg[k2];
    nU -= e.count;
    eU -= (long long)e.in_edges;
    const int v = device_decides ? e.variant : host_variant[k2];
    if (st->level_variant) st->level_variant[k2] = v;
    if (st->level_frontier) st->level_frontier[k2] = e.count;
    if (st->level_frontier_edges) st->level_frontier_edges[k2] = (int64_t)e.edges;
    if (st->level_unvisited) st->level_unvisited[k2] = nU;
    if (st->level_unvisited_edges) st->level_unvisited_edges[k2] = eU;
    if (st->level_fallback) st->level_fallback[k2] = e.fallback;
    if (st->level_frontier_ld) st->level_frontier_ld[k2] = (int64_t)e.ld;
    if (st->level_frontier_ld2) st->level_frontier_ld2[k2] = (int64_t)e.ld2;
    if (st->level_scanned) st->level_scanned[k2] = (int64_t)lg[k2 + 1].scanned;
    if (st->level_next) st->level_next[k2] = lg[k2 + 1].count;
    float lms = (timing && k2 < (int)level_ms.size()) ? level_ms[k2] : 0.f;
    if (timing && persistent && k2 + 1 < L) lms = (float)((double)(lg[k2 + 1].t - lg[k2].t) / wall_khz());
    if (st->level_ms) st->level_ms[k2] = lms;
  }
  return BFS_OK;
}

// Exact state of level k from finished depths, then `reps` timed steps.
static int step_time(const bfs_graph *g, const int *depths, int k, int variant, int reps, int *scratch,
                     const bfs_options *opt, float *ms_out, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!depths || !scratch || !ms_out || reps <= 0 || k < 0 || variant < 0 || variant >= BFS_NUM_VARIANTS) {
    set_error("invalid bfs_step_time arguments");
    return BFS_EINVAL;
  }
  if (opt && opt->vertex_map) {
    set_error("options.vertex_map is not honoured by bfs_step_time");
    return BFS_ENOTSUP;
  }
  if (is_pull(variant) && !g->csc_ptr) {
    set_error("pull variant needs CSC arrays");
    return BFS_ENOTSUP;
  }
  HostCtx &hc = host_ctx();
  const size_t need = workspace_bytes_single(g->n);
  void *wsp = opt ? opt->workspace : nullptr;
  if (wsp) {
    if (opt->workspace_bytes < need) return BFS_EWORKSPACE;
  } else {
    rc = cached_workspace(need, &wsp);
    if (rc) return rc;
  }
  Workspace w = carve_single(wsp, g->n);
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    StepArgs a = level_args(g, w, scratch, nullptr, k, DEFAULT_HUB);
    BFS_HIP(launch_state_from_depths(a, depths, w.ring, s));
    BFS_HIP(hipMemcpyAsync(hc.pinned, a.c_cur, sizeof(LevelCtr), hipMemcpyDeviceToHost, s));
    BFS_HIP(hipStreamSynchronize(s));
    long long cnt = hc.pinned[0].count, eF = (long long)hc.pinned[0].edges;
    a.hub = hub_threshold(cnt);
    BFS_HIP(hipEventRecord(hc.ev[0], s));
    BFS_HIP(launch_step(variant, a, (int)cnt, eF, s));
    BFS_HIP(hipEventRecord(hc.ev[1], s));
    BFS_HIP(hipEventSynchronize(hc.ev[1]));
    float ms = 0.f;
    BFS_HIP(hipEventElapsedTime(&ms, hc.ev[0], hc.ev[1]));
    t.push_back(ms);
  }
  std::sort(t.begin(), t.end());
  *ms_out = t[t.size() / 2];
  return BFS_OK;
}

// ------------------------------------------------- allocation-free search
// bfs_levels_noalloc's scratch: a file-scope device array in place of a
// workspace, for callers that cannot allocate (graph capture, serving loops).
// Each GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {nullptr};

static int scratch_address(void **out) {
  int dev = 0;
  BFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device %d out of range", dev);
    return BFS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BFS_OK;
}

// Largest n whose single-source workspace fits in the scratch array.
static int noalloc_max_n() {
  int lo = 1, hi = 1 << 26;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (workspace_bytes_single(mid) <= NOALLOC_SCRATCH_BYTES) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Zero-fill of device words (a kernel, not a memset node, so a captured
// stream replays it correctly).
__global__ void k_fill0(u64 *p, int words) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

// Device-to-host copy of a few bytes into host stack memory, then a stream
// synchronisation: no pinned staging buffer of the library's own.
static int read_back(void *dst, const void *src, size_t bytes, hipStream_t s) {
  BFS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  return BFS_OK;
}

// The search of run_single on the scratch array, with every level choice
// made on the device: the step kernels for the next levels are enqueued in
// batches, each gated by the decision and frontier size of its level, and the
// host reads the loop control once per batch.  Depths only; per-level
// statistics and level timing are not offered here.
static int run_single_noalloc(const bfs_graph *g, int src, int *levels, const bfs_options *opt_in, bfs_stats *st,
                              hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!levels) {
    set_error("levels is NULL");
    return BFS_EINVAL;
  }
  if (src < 0 || src >= g->n) {
    set_error("source %d out of range [0, %d)", src, g->n);
    return BFS_EINVAL;
  }
  const int max_n = noalloc_max_n();
  if (g->n > max_n) {
    set_error("bfs_levels_noalloc: n = %d exceeds the %d vertices its %zu-byte scratch holds", g->n, max_n,
              NOALLOC_SCRATCH_BYTES);
    return BFS_EWORKSPACE;
  }
  bfs_options dflt;
  memset(&dflt, 0, sizeof(dflt));
  dflt.variant = selector_loaded() ? BFS_AUTO_LEARNED : BFS_AUTO_HEURISTIC;
  dflt.heuristic_push = -1;
  dflt.heuristic_pull = -1;
  const bfs_options *opt = opt_in ? opt_in : &dflt;
  if (opt->flags & (BFS_F_LEVEL_STATS | BFS_F_LEVEL_TIMING | BFS_F_DEVICE_LOOP)) {
    set_error("bfs_levels_noalloc: per-level statistics, level timing and the persistent loop are not offered");
    return BFS_ENOTSUP;
  }
  int mode = opt->variant;
  const bool have_csc = g->csc_ptr != nullptr;
  if (mode >= 0 && mode < BFS_NUM_VARIANTS) {
    if (is_pull(mode) && !have_csc) {
      set_error("pull variant needs CSC arrays");
      return BFS_ENOTSUP;
    }
  } else if (mode == BFS_SCHEDULE) {
    if (!opt->schedule_host || opt->schedule_len <= 0) {
      set_error("BFS_SCHEDULE needs schedule_host and schedule_len > 0");
      return BFS_EINVAL;
    }
    for (int i = 0; i < opt->schedule_len; ++i) {
      const int v = opt->schedule_host[i];
      if (v < 0 || v >= BFS_NUM_VARIANTS || (is_pull(v) && !have_csc)) {
        set_error("schedule entry %d is not a usable variant", i);
        return v < 0 || v >= BFS_NUM_VARIANTS ? BFS_EINVAL : BFS_ENOTSUP;
      }
    }
  } else if (mode != BFS_AUTO_HEURISTIC && mode != BFS_AUTO_LEARNED) {
    set_error("unknown variant/mode %d", mode);
    return BFS_EINVAL;
  }
  bool learned = mode == BFS_AUTO_LEARNED;
  int fell_back_all = 0;
  if (learned && !selector_loaded()) {
    if (opt->flags & BFS_F_STRICT_SELECTOR) {
      set_error("learned mode requested but no selector weights are loaded");
      return BFS_ENOSEL;
    }
    learned = false;
    mode = BFS_AUTO_HEURISTIC;
    fell_back_all = 1;
  }
  const bool device_decides = mode == BFS_AUTO_HEURISTIC || mode == BFS_AUTO_LEARNED;
  const int push_v = (opt->heuristic_push >= 0 && opt->heuristic_push < BFS_NUM_VARIANTS &&
                      !is_pull(opt->heuristic_push)) ? opt->heuristic_push : BFS_V_PUSH_Q_BLOCK;
  const int pull_v = have_csc ? BFS_V_PULL_B : push_v;
  void *wsp = nullptr;
  rc = scratch_address(&wsp);
  if (rc) return rc;
  Workspace w = carve_single(wsp, g->n);
  const auto t0 = std::chrono::steady_clock::now();
  int syncs = 0;
  if (opt->flags & BFS_F_VALIDATE) {
    u64 *flag = w.gsum + 8;
    hipLaunchKernelGGL(k_fill0, dim3(1), dim3(64), 0, s, flag, 1);
    BFS_HIP(launch_validate(g->n, g->nnz, g->row_ptr, g->col_idx, flag, s));
    if (g->csc_ptr && g->csc_ptr != g->row_ptr) BFS_HIP(launch_validate(g->n, g->nnz, g->csc_ptr, g->csc_idx, flag, s));
    u64 bad = 0;
    rc = read_back(&bad, flag, 8, s);
    if (rc) return rc;
    ++syncs;
    if (bad) {
      set_error("malformed graph: %s%s", (bad & 1) ? "bad offsets " : "", (bad & 2) ? "column id out of range" : "");
      return BFS_EGRAPH;
    }
  }
  const int *vmap = opt->vertex_map;
  int *levels_out = levels;
  const MapBufs mb = map_bufs(wsp, g->n);
  if (vmap) {
    int nsrc = -1;
    rc = read_back(&nsrc, vmap + src, sizeof(int), s);
    if (rc) return rc;
    ++syncs;
    if (nsrc < 0 || nsrc >= g->n) {
      set_error("vertex_map maps the source to %d, outside [0, %d)", nsrc, g->n);
      return BFS_EINVAL;
    }
    src = nsrc;
    levels = mb.lv;
  }
  const long long maxlev = opt->max_levels > 0 ? opt->max_levels : (long long)g->n + 1;
  u64 gld = 0, gld2 = 0;
  if (learned) {
    if (opt->flags & BFS_F_GRAPH_SUMS) {
      gld = (u64)opt->graph_ld;
      gld2 = (u64)opt->graph_ld2;
    } else {
      BFS_HIP(launch_graph_ld(g->n, g->row_ptr, w.gsum, s));
      u64 sums[2] = {0, 0};
      rc = read_back(sums, w.gsum, 16, s);
      if (rc) return rc;
      ++syncs;
      gld = sums[0];
      gld2 = sums[1];
    }
  }
  int cands[2 + NC];  // the variants a device-decided level may run
  int ncand = 0;
  if (device_decides) {
    cands[ncand++] = push_v;
    if (pull_v != push_v) cands[ncand++] = pull_v;
    if (learned) {
      SelDevice probe = selector_device(w, push_v, pull_v);
      for (int c = 0; c < NC; ++c) {
        const int v = probe.cls[c];
        if (is_pull(v) && !have_csc) continue;
        if (std::find(cands, cands + ncand, v) == cands + ncand) cands[ncand++] = v;
      }
    }
  }
  hipLaunchKernelGGL(k_fill0, dim3(1), dim3(64), 0, s, reinterpret_cast<u64 *>(w.ctl), (int)(sizeof(LoopCtl) / 8));
  StepArgs a = level_args(g, w, levels, nullptr, 0, DEFAULT_HUB);
  SelDevice seldev = selector_device(w, push_v, pull_v);
  seldev.gld = gld;
  seldev.gld2 = gld2;
  BFS_HIP(launch_reset(a, src, w.ring, s));
  BFS_HIP(launch_finish_f0(w, s));
  if (device_decides) BFS_HIP(launch_select(seldev, w.ring, 0, g->n, g->nnz, s, true, learned, w.log));
  constexpr int BATCH = 16;
  LoopCtl ctl;
  memset(&ctl, 0, sizeof(ctl));
  int k = 0;
  for (bool done = false; !done;) {
    for (int i = 0; i < BATCH; ++i, ++k) {
      a = level_args(g, w, levels, nullptr, k, DEFAULT_HUB);
      if (device_decides) {
        for (int c = 0; c < ncand; ++c) {
          a.gate = cands[c];
          BFS_HIP(launch_step(cands[c], a, -1, -1, s));
        }
      } else {
        a.gate = -2;
        const int v = mode == BFS_SCHEDULE ? opt->schedule_host[std::min(k, opt->schedule_len - 1)] : mode;
        BFS_HIP(launch_step(v, a, -1, -1, s));
      }
      BFS_HIP(launch_finish_select(&w.ring[(k + 1) % RING], w.qcap, k + 1, w.log, w.ctl, seldev, w.ring, g->n, g->nnz,
                                   device_decides, learned, nullptr, nullptr, 0, s));
    }
    rc = read_back(&ctl, w.ctl, sizeof(LoopCtl), s);
    if (rc) return rc;
    ++syncs;
    done = ctl.done != 0;
    if (!done && k >= maxlev) {
      set_error("level loop reached max_levels = %lld", maxlev);
      return BFS_ELEVELCAP;
    }
  }
  if ((long long)ctl.levels > maxlev) {
    set_error("level loop reached max_levels = %lld", maxlev);
    return BFS_ELEVELCAP;
  }
  if (vmap) {
    const int grid = std::min(4096, (g->n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_unmap, dim3(grid), dim3(BLOCK), 0, s, vmap, (const int *)nullptr, (const int *)mb.lv,
                       (const int *)nullptr, levels_out, (int *)nullptr, g->n);
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipStreamSynchronize(s));
    ++syncs;
  }
  if (st) {
    st->num_levels = (int)ctl.levels;
    st->reached = (int64_t)ctl.reached;
    st->component_edges = (int64_t)ctl.comp_edges;
    st->elapsed_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st->host_syncs = syncs;
    st->fell_back = fell_back_all;
  }
  return BFS_OK;
}

}  // namespace bfs

// ------------------------------------------------------------------ C ABI
using namespace bfs;

extern "C" {

const char *bfs_strerror(int code) {
  switch (code) {
    case BFS_OK: return "ok";
    case BFS_EINVAL: return "invalid argument";
    case BFS_EGRAPH: return "malformed graph";
    case BFS_EWORKSPACE: return "workspace too small";
    case BFS_EHIP: return "HIP runtime error";
    case BFS_ENOSEL: return "no selector weights loaded";
    case BFS_ELEVELCAP: return "level cap reached";
    case BFS_ENOTSUP: return "variant not supported for this graph";
    case BFS_EFILE: return "selector weights file missing or malformed";
    default: return "unknown error";
  }
}

const char *bfs_last_error(void) { return g_err; }

int bfs_version(void) { return 1; }

int bfs_workspace_size(int32_t n, int32_t lanes, size_t *bytes) {
  if (n <= 0 || !bytes || lanes < 1 || lanes > 64) {
    set_error("invalid bfs_workspace_size arguments");
    return BFS_EINVAL;
  }
  *bytes = lanes == 1 ? workspace_bytes_single(n) : workspace_bytes_multi(n);
  return BFS_OK;
}

int bfs_levels(const bfs_graph *g, int32_t source, int32_t *levels, const bfs_options *opt, bfs_stats *st,
               void *stream) {
  if (!levels) {
    set_error("levels is NULL");
    return BFS_EINVAL;
  }
  return run_single(g, source, levels, nullptr, opt, st, (hipStream_t)stream);
}

int bfs_parents(const bfs_graph *g, int32_t source, int32_t *levels, int32_t *parents, const bfs_options *opt,
                bfs_stats *st, void *stream) {
  if (!levels || !parents) {
    set_error("levels or parents is NULL");
    return BFS_EINVAL;
  }
  return run_single(g, source, levels, parents, opt, st, (hipStream_t)stream);
}

int bfs_levels_noalloc(const bfs_graph *g, int32_t source, int32_t *levels, const bfs_options *opt, bfs_stats *st,
                       void *stream) {
  return run_single_noalloc(g, source, levels, opt, st, (hipStream_t)stream);
}

int bfs_graph_sums(const bfs_graph *g, int64_t *ld, int64_t *ld2, void *stream) {
  if (!g || g->n <= 0 || !g->row_ptr || !ld || !ld2) {
    set_error("bfs_graph_sums: invalid argument");
    return BFS_EINVAL;
  }
  static std::mutex mu;
  static u64 *buf[64] = {nullptr};
  int dev = 0;
  BFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) dev = 0;
  Workspace w{};
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!buf[dev]) BFS_HIP(hipMalloc((void **)&buf[dev], GSUM_WORDS * 8));
    w.gsum = buf[dev];
  }
  u64 a = 0, b = 0;
  const int rc = graph_ld_sums(g, w, (hipStream_t)stream, &a, &b);
  if (rc) return rc;
  *ld = (int64_t)a;
  *ld2 = (int64_t)b;
  return BFS_OK;
}

int bfs_step_time(const bfs_graph *g, const int32_t *depths, int32_t k, int32_t variant, int32_t reps,
                  int32_t *scratch_levels, const bfs_options *opt, float *ms_out, void *stream) {
  return step_time(g, depths, k, variant, reps, scratch_levels, opt, ms_out, (hipStream_t)stream);
}

}  // extern "C"
