// Selector network kernels: device-side per-level selection (inference on one
// feature vector), batched forward, loss/gradient and Adam for training.
//
// Network: x (12 normalised features) -> h0 = bf16(x)
//   z1 = b1 + W1 h0, h1 = bf16(relu(z1))
//   z2 = b2 + W2 h1, h2 = bf16(relu(z2))
//   logits = b3 + W3 h2
// with W = bf16(W_master).  Each output is accumulated in fp32 starting from
// its bias, adding products in ascending input order.  A product of two bf16
// values is exact in fp32, so a fused multiply-add gives the same result as a
// separate multiply and add; the order is what makes the result reproducible.
// Backward treats each bf16 rounding as the identity (straight-through).
#include <stdio.h>
#include <string.h>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "selector.hpp"
#include "selector_dev.hpp"
#include "step_bodies.hpp"

namespace bfs {

__global__ __launch_bounds__(64) void k_select(SelDevice sd, RingSlot *ring, int k, int n, int nnz, int init,
                                               int use_net, LevelLog *log) {
  __shared__ __align__(16) char smem[SM_SELECT];
  if (use_net) {
    NetRegs nr;
    load_net(sd, nr);
    body_select<true>(sd, ring, k, n, nnz, init, use_net, log, smem, nr);
  } else {
    body_select(sd, ring, k, n, nnz, init, use_net, log, smem);
  }
}

// The per-level counter reduction followed, in the same workgroup, by the
// choice for the next level (when `select`): one launch per level instead of
// two.  With `host` (pinned host memory) the level's totals, decision
// included, are also copied there, and then -- after a system-scope fence --
// `seq` is written to *host_seq for the host loop to poll.
// The work is that of body_finish then body_select (the same values are
// written: segment offsets, totals, log entry, loop control, selector state,
// decision), arranged for latency, as this launch sits between two steps on
// the host loop's critical path: every global load it needs (the shards, the
// loop control, the selector state, and for the network this lane's weight
// rows and its feature's normalisation) is issued at the start, the totals
// and state then travel through registers and LDS instead of being written
// and read back, and the host copy is written from registers.
__global__ __launch_bounds__(NSH) void k_finish_select(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl,
                                                       SelDevice sd, RingSlot *ring, int n, int nnz, int select,
                                                       int use_net, LevelCtr *host, u64 *host_seq, u64 seq) {
  (void)ring;  // slot is ring[k % RING]
  __shared__ u64 s_red[5][NSH / WAVE];
  __shared__ int s_w[NSH / WAVE];
  __shared__ __align__(16) float s_net[NF + 3 * NH];
  __shared__ u64 s_tot[4];      // count, edges, ld, ld2 of F_k
  __shared__ long long s_u[2];  // nU, eU after F_k
  __shared__ int s_hv;
  const int t = threadIdx.x;
  const bool net = select && use_net;
  long long *st = reinterpret_cast<long long *>(sd.state);
  // loads first
  const LevelCtr c = slot->sh[t];
  u32 ovf = 0;
  u64 done = 0, reached = 0, comp = 0;
  long long st0 = 0, st1 = 0, st2 = 0, st3 = 0;
  if (t == 0) {
    ovf = slot->sh[NSH].count;
    done = ctl->done;
    reached = ctl->reached;
    comp = ctl->comp_edges;
    if (select) {
      st0 = st[0];
      st1 = st[1];
      st2 = st[2];
      st3 = st[3];
    }
  }
  NetRegs nr;
  float nmean = 0.f, nstd = 1.f, nmin = 0.f, nmax = 0.f;
  if (net && t < WAVE) {
    load_net(sd, nr);
    if (t < NF) {
      nmean = sd.norm[t];
      nstd = sd.norm[NF + t];
      nmin = sd.norm[2 * NF + t];
      nmax = sd.norm[3 * NF + t];
    }
  }
  // counter reduction and queue segment offsets (body_finish)
  const int cnt = (int)min(c.count, (u32)qcap);
  const int w = t / WAVE;
  const int incl = wave_incl_scan(cnt);
  if (lane() == WAVE - 1) s_w[w] = incl;
  const u64 v[5] = {c.edges, c.in_edges, c.ld, c.ld2, c.scanned};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const u64 r = wave_sum_u64(v[j]);
    if (lane() == 0) s_red[j][w] = r;
  }
  __syncthreads();
  int off = 0, total = 0;
  for (int i = 0; i < NSH / WAVE; ++i) {
    off += (i < w) ? s_w[i] : 0;
    total += s_w[i];
  }
  slot->seg[t] = off + incl - cnt;
  LevelCtr o;  // thread 0: the totals of F_k
  int hv = -1;
  if (t == 0) {
    u64 r[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < 5; ++j)
      for (int i = 0; i < NSH / WAVE; ++i) r[j] += s_red[j][i];
    o.count = (u32)(total + (int)ovf);
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
    slot->seg[NSH] = total;
    slot->seg[NSH + 1] = total + (int)ovf;
    if (o.count == 0) {
      ctl->done = 1;
    } else if (!done) {
      ctl->levels = (u64)k + 1;
      ctl->reached = reached + o.count;
      ctl->comp_edges = comp + o.edges;
    }
    if (select) {  // the unvisited totals after F_k and the direction rule (body_select)
      const long long nF = o.count;
      st0 -= nF;
      st1 -= (long long)o.in_edges;
      const long long eF = (long long)o.edges, eU = st1;
      int dir = (int)st2;
      if (dir == 0) {
        if (eF * HeuristicState::kAlpha > eU) dir = 1;
      } else {
        const bool shrinking = st3 >= 0 && nF < st3;
        if (nF * HeuristicState::kBeta < (long long)n && shrinking) dir = 0;
      }
      st[0] = st0;
      st[1] = st1;
      st[2] = dir;
      st[3] = nF;
      hv = dir ? sd.pull_v : sd.push_v;
      s_u[0] = st0;
      s_u[1] = st1;
      s_hv = hv;
      s_tot[0] = o.count;
      s_tot[1] = o.edges;
      s_tot[2] = o.ld;
      s_tot[3] = o.ld2;
    }
  }
  int dec = -1, fb = 0;
  if (net) {
    __syncthreads();  // uniform: the totals and state are in LDS
    if (t < WAVE) {
      hv = s_hv;
      dec = hv;
      // the level's raw features, one per lane; range check, then normalise
      bool out_of_range = false;
      float xn = 0.f;
      if (lane() < NF) {
        const float r = level_feature(lane(), (double)n, (double)nnz, (double)k, (double)s_tot[0],
                                      (double)s_tot[1], (double)s_u[0], (double)s_u[1], (double)s_tot[2],
                                      (double)s_tot[3], (double)sd.gld, (double)sd.gld2);
        out_of_range = r < nmin || r > nmax;
        xn = (r - nmean) / nstd;
      }
      const bool any_oor = __ballot(out_of_range) != 0ull;
      float *s_x = s_net, *h0 = s_net + NF, *h1 = h0 + NH, *h2 = h1 + NH;
      if (lane() < NF) s_x[lane()] = xn;
      __builtin_amdgcn_wave_barrier();
      const float logit = forward_row_regs(nr, s_x, h0, h1, h2);
      int cls;
      float conf;
      argmax_conf(logit, &cls, &conf);
      fb = any_oor || !(conf >= sd.min_conf);
      dec = fb ? hv : sd.cls[cls];
    }
  } else if (select) {
    dec = hv;  // thread 0: the direction rule's choice
  }
  if (t == 0) {
    o.decision = select ? dec : -1;
    o.fallback = select ? fb : 0;
    slot->tot = o;
    if (k < LOGCAP) {
      LevelLog &L = log[k];
      L.count = o.count;
      L.variant = o.decision;
      L.edges = o.edges;
      L.in_edges = o.in_edges;
      L.ld = o.ld;
      L.ld2 = o.ld2;
      L.scanned = o.scanned;
      L.fallback = o.fallback;
    }
    if (host) {
      *host = o;
      __threadfence_system();
      *reinterpret_cast<volatile u64 *>(host_seq) = seq;
    }
  }
}

// Level 0 of the host loop in one launch: F_0 = {src} into slot 0 (its
// totals and queue segment offsets, as k_reset_f0 writes them), its log
// entry and the loop control (as k_log_f0), the choice for level 0 when
// `select` (the selector state initialised and the direction rule applied,
// then the network, as body_select with init), and the totals posted to
// host memory as k_finish_select does.  One wave; k_reset has cleared the
// ring.
__global__ __launch_bounds__(WAVE) void k_start_select(const int *rp, const int *cp, int src, RingSlot *slot0,
                                                       LevelLog *log, LoopCtl *ctl, SelDevice sd, int n, int nnz,
                                                       int select, int use_net, LevelCtr *host, u64 *host_seq,
                                                       u64 seq) {
  __shared__ __align__(16) float s_net[NF + 3 * NH];
  const int l = lane();
  const bool net = select && use_net;
  NetRegs nr;
  float nmean = 0.f, nstd = 1.f, nmin = 0.f, nmax = 0.f;
  if (net) {
    load_net(sd, nr);
    if (l < NF) {
      nmean = sd.norm[l];
      nstd = sd.norm[NF + l];
      nmin = sd.norm[2 * NF + l];
      nmax = sd.norm[3 * NF + l];
    }
  }
  for (int i = l; i < NSH + 2; i += WAVE) slot0->seg[i] = (i == 0) ? 0 : 1;
  const int d = rp[src + 1] - rp[src];
  const int di = cp ? cp[src + 1] - cp[src] : d;
  const int lg = ilog2p1(d);
  LevelCtr o;
  o.count = 1;
  o.nhub = 0;
  o.edges = (u64)d;
  o.in_edges = (u64)di;
  o.ld = (u64)lg;
  o.ld2 = (u64)(lg * lg);
  o.scanned = 0;
  o.ntiles = 0;
  o.total_e = 0;
  int dec = -1, fb = 0;
  if (select) {
    // selector state after F_0 = {src}: nU = n - 1, eU = nnz - in-degree,
    // and the direction rule from top-down with no previous frontier
    const long long nU = (long long)n - 1, eU = (long long)nnz - di;
    const int dir = (long long)d * HeuristicState::kAlpha > eU ? 1 : 0;
    if (l == 0) {
      long long *st = reinterpret_cast<long long *>(sd.state);
      st[0] = nU;
      st[1] = eU;
      st[2] = dir;
      st[3] = 1;
    }
    const int hv = dir ? sd.pull_v : sd.push_v;
    dec = hv;
    if (net) {
      bool out_of_range = false;
      float xn = 0.f;
      if (l < NF) {
        const float r = level_feature(l, (double)n, (double)nnz, 0.0, 1.0, (double)d, (double)nU, (double)eU,
                                      (double)lg, (double)(lg * lg), (double)sd.gld, (double)sd.gld2);
        out_of_range = r < nmin || r > nmax;
        xn = (r - nmean) / nstd;
      }
      const bool any_oor = __ballot(out_of_range) != 0ull;
      float *s_x = s_net, *h0 = s_net + NF, *h1 = h0 + NH, *h2 = h1 + NH;
      if (l < NF) s_x[l] = xn;
      __builtin_amdgcn_wave_barrier();
      const float logit = forward_row_regs(nr, s_x, h0, h1, h2);
      int cls;
      float conf;
      argmax_conf(logit, &cls, &conf);
      fb = any_oor || !(conf >= sd.min_conf);
      dec = fb ? hv : sd.cls[cls];
    }
  }
  if (l == 0) {
    o.decision = dec;
    o.fallback = fb;
    slot0->tot = o;
    LevelLog &L = log[0];
    L.count = 1;
    L.variant = dec;
    L.edges = o.edges;
    L.in_edges = o.in_edges;
    L.ld = o.ld;
    L.ld2 = o.ld2;
    L.scanned = 0;
    L.fallback = fb;
    ctl->done = 0;
    ctl->levels = 1;
    ctl->reached = 1;
    ctl->comp_edges = o.edges;
    if (host) {
      *host = o;
      __threadfence_system();
      *reinterpret_cast<volatile u64 *>(host_seq) = seq;
    }
  }
}

hipError_t launch_start_select(const int *rp, const int *cp, int src, RingSlot *slot0, LevelLog *log, LoopCtl *ctl,
                               const SelDevice &sd, int n, int nnz, bool select, bool use_net, LevelCtr *host,
                               u64 *host_seq, u64 seq, hipStream_t s) {
  hipLaunchKernelGGL(k_start_select, dim3(1), dim3(WAVE), 0, s, rp, cp, src, slot0, log, ctl, sd, n, nnz,
                     select ? 1 : 0, (use_net && sd.use_net) ? 1 : 0, host, host_seq, seq);
  return hipGetLastError();
}

hipError_t launch_finish_select(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl, const SelDevice &sd,
                                RingSlot *ring, int n, int nnz, bool select, bool use_net, LevelCtr *host,
                                u64 *host_seq, u64 seq, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_select, dim3(1), dim3(NSH), 0, s, slot, qcap, k, log, ctl, sd, ring, n, nnz,
                     select ? 1 : 0, (use_net && sd.use_net) ? 1 : 0, host, host_seq, seq);
  return hipGetLastError();
}

// ------------------------------------------------------------ selector set
struct SelectorHost {
  bool loaded = false;
  int dev = -1;
  void *buf = nullptr;  // [bf16 weights NPARAM u16 | fp32 params NPARAM | norm 4*NF]
  float min_conf = 0.f;
  int cls[NC] = {0, 1, 2, 3};
};
static std::mutex g_sel_mu;
static SelectorHost g_sel[64];

static int cur_dev() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return 0;
  return (d >= 0 && d < 64) ? d : 0;
}

bool selector_loaded() {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  return g_sel[cur_dev()].loaded;
}

SelDevice selector_device(const Workspace &w, int push_v, int pull_v) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  SelectorHost &h = g_sel[cur_dev()];
  SelDevice d;
  d.use_net = h.loaded && h.buf;
  char *b = (char *)h.buf;
  d.w = (const u16 *)b;
  d.p = (const float *)(b + ((NPARAM * 2 + 255) & ~255));
  d.norm = d.p + NPARAM;
  d.min_conf = h.min_conf;
  for (int i = 0; i < NC; ++i) d.cls[i] = h.cls[i];
  d.state = w.gsum + 2;
  d.push_v = push_v;
  d.pull_v = pull_v;
  d.gld = d.gld2 = 0;
  return d;
}

hipError_t launch_select(const SelDevice &sd, RingSlot *ring, int k, int n, int nnz, hipStream_t s, bool init,
                         bool use_net, LevelLog *log) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, sd, ring, k, n, nnz, init ? 1 : 0,
                     (use_net && sd.use_net) ? 1 : 0, log);
  return hipGetLastError();
}

// ---------------------------------------------------------- training kernels
constexpr int MLP_BLOCK = 256;  // 4 waves, one row per wave at a time

__global__ __launch_bounds__(MLP_BLOCK) void k_mlp_forward(const float *p, const float *x, int batch,
                                                           float *logits, int *cls, float *conf) {
  __shared__ float s_h[MLP_BLOCK / WAVE][3][NH];
  const int wv = threadIdx.x / WAVE;
  float *h0 = s_h[wv][0], *h1 = s_h[wv][1], *h2 = s_h[wv][2];
  for (int r = blockIdx.x * (MLP_BLOCK / WAVE) + wv; r < batch; r += gridDim.x * (MLP_BLOCK / WAVE)) {
    float z1, z2;
    float lg = forward_row(WMaster{p}, p, x + (size_t)r * NF, h0, h1, h2, z1, z2);
    if (logits && lane() < NC) logits[(size_t)r * NC + lane()] = lg;
    if (cls) {
      int c;
      float cf;
      argmax_conf(lg, &c, &cf);
      if (lane() == 0) {
        cls[r] = c;
        conf[r] = cf;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Gradient of mean cross-entropy.  A workgroup handles rows in turn: wave 0
// computes the row's forward and backward vectors into LDS, then all 256
// threads add the row's outer products into privately owned gradient slots;
// at the end each owned slot is added to the global gradient once.
constexpr int GRAD_ROWS = 64;
__global__ __launch_bounds__(MLP_BLOCK) void k_mlp_grad(const float *p, const float *x, const int *labels,
                                                        int batch, float *grad, float *loss) {
  __shared__ float h0[NH], h1[NH], h2[NH], dz1[NH], dz2[NH], dl[NC];
  __shared__ float s_loss;
  constexpr int PER = (NPARAM + MLP_BLOCK - 1) / MLP_BLOCK;  // owned slots per thread
  float acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) acc[i] = 0.f;
  if (threadIdx.x == 0) s_loss = 0.f;
  const float invB = 1.f / (float)batch;
  const int r0 = blockIdx.x * GRAD_ROWS;
  const int r1 = min(batch, r0 + GRAD_ROWS);
  for (int r = r0; r < r1; ++r) {
    if (threadIdx.x < WAVE) {
      const int l = lane();
      float z1, z2;
      float lg = forward_row(WMaster{p}, p, x + (size_t)r * NF, h0, h1, h2, z1, z2);
      float L0 = __shfl(lg, 0), L1 = __shfl(lg, 1), L2 = __shfl(lg, 2), L3 = __shfl(lg, 3);
      float mx = fmaxf(fmaxf(L0, L1), fmaxf(L2, L3));
      float e0 = expf(L0 - mx), e1 = expf(L1 - mx), e2 = expf(L2 - mx), e3 = expf(L3 - mx);
      float se = e0 + e1 + e2 + e3;
      const int y = labels[r];
      if (l < NC) {
        float pj = (l == 0 ? e0 : l == 1 ? e1 : l == 2 ? e2 : e3) / se;
        dl[l] = (pj - (l == y ? 1.f : 0.f)) * invB;
      }
      if (l == 0) {
        float ly = (y == 0 ? L0 : y == 1 ? L1 : y == 2 ? L2 : L3);
        s_loss += (logf(se) + mx - ly) * invB;
      }
      __builtin_amdgcn_wave_barrier();
      // dh2[l] = sum_j dl[j] * W3r[j][l]; dz2 = dh2 * (z2 > 0)
      float d2 = 0.f;
      for (int j = 0; j < NC; ++j) d2 += dl[j] * bfr(p[OFF_W3 + j * NH + l]);
      d2 = (z2 > 0.f) ? d2 : 0.f;
      dz2[l] = d2;
      __builtin_amdgcn_wave_barrier();
      float d1 = 0.f;
      for (int j = 0; j < NH; ++j) d1 += dz2[j] * bfr(p[OFF_W2 + j * NH + l]);
      d1 = (z1 > 0.f) ? d1 : 0.f;
      dz1[l] = d1;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * MLP_BLOCK;
      if (q >= NPARAM) break;
      float gq;
      if (q < OFF_B1) gq = dz1[q / NF] * h0[q % NF];
      else if (q < OFF_W2) gq = dz1[q - OFF_B1];
      else if (q < OFF_B2) gq = dz2[(q - OFF_W2) / NH] * h1[(q - OFF_W2) % NH];
      else if (q < OFF_W3) gq = dz2[q - OFF_B2];
      else if (q < OFF_B3) gq = dl[(q - OFF_W3) / NH] * h2[(q - OFF_W3) % NH];
      else gq = dl[q - OFF_B3];
      acc[i] += gq;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int q = threadIdx.x + i * MLP_BLOCK;
    if (q < NPARAM && acc[i] != 0.f) atomicAdd(grad + q, acc[i]);
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, s_loss);
}

__global__ void k_mlp_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
  }
}

}  // namespace bfs

using namespace bfs;

extern "C" {

int bfs_selector_set(const float *params, const float *mean, const float *stdv, const float *fmin,
                     const float *fmax, float min_confidence, const int32_t *class_variant) {
  if (!params || !mean || !stdv || !fmin || !fmax || !class_variant) {
    set_error("bfs_selector_set: null argument");
    return BFS_EINVAL;
  }
  for (int i = 0; i < NC; ++i)
    if (class_variant[i] < 0 || class_variant[i] >= BFS_NUM_VARIANTS) {
      set_error("bfs_selector_set: class %d maps to invalid variant %d", i, class_variant[i]);
      return BFS_EINVAL;
    }
  for (int i = 0; i < NF; ++i)
    if (!(stdv[i] > 0.f)) {
      set_error("bfs_selector_set: feature std %d is not positive", i);
      return BFS_EINVAL;
    }
  const size_t wbytes = (NPARAM * 2 + 255) & ~(size_t)255;
  const size_t total = wbytes + (NPARAM + 4 * NF) * sizeof(float);
  std::vector<char> host(total, 0);
  u16 *w = (u16 *)host.data();
  float *p = (float *)(host.data() + wbytes);
  for (int i = 0; i < NPARAM; ++i) {
    w[i] = f2bf(params[i]);
    p[i] = params[i];
  }
  float *norm = p + NPARAM;
  memcpy(norm, mean, NF * 4);
  memcpy(norm + NF, stdv, NF * 4);
  memcpy(norm + 2 * NF, fmin, NF * 4);
  memcpy(norm + 3 * NF, fmax, NF * 4);
  std::lock_guard<std::mutex> lk(g_sel_mu);
  SelectorHost &h = g_sel[cur_dev()];
  if (!h.buf) BFS_HIP(hipMalloc(&h.buf, total));
  BFS_HIP(hipMemcpy(h.buf, host.data(), total, hipMemcpyHostToDevice));
  h.min_conf = min_confidence;
  for (int i = 0; i < NC; ++i) h.cls[i] = class_variant[i];
  h.loaded = true;
  return BFS_OK;
}

// Weights file (little-endian; layout in bfs_eeds.h): parsed and checked in
// full on the host before anything reaches the device.
int bfs_selector_load(const char *path) {
  if (!path) {
    set_error("bfs_selector_load: path is NULL");
    return BFS_EINVAL;
  }
  FILE *f = fopen(path, "rb");
  if (!f) {
    set_error("bfs_selector_load: cannot open %s", path);
    return BFS_EFILE;
  }
  constexpr size_t kFloats = NPARAM + 4 * NF + 1;
  constexpr size_t kBytes = 24 + kFloats * 4 + NC * 4;
  std::vector<unsigned char> buf(kBytes + 1);
  const size_t got = fread(buf.data(), 1, buf.size(), f);
  fclose(f);
  if (got != kBytes) {
    set_error("bfs_selector_load: %s holds %zu bytes, expected %zu", path, got, kBytes);
    return BFS_EFILE;
  }
  auto rd32 = [&](size_t off) {
    return (uint32_t)buf[off] | ((uint32_t)buf[off + 1] << 8) | ((uint32_t)buf[off + 2] << 16) |
           ((uint32_t)buf[off + 3] << 24);
  };
  if (memcmp(buf.data(), "BFSSEL01", 8) != 0 || rd32(8) != 1u || rd32(12) != (uint32_t)NPARAM ||
      rd32(16) != (uint32_t)NF || rd32(20) != (uint32_t)NC) {
    set_error("bfs_selector_load: %s is not a version-1 selector file for a 12-64-64-4 network", path);
    return BFS_EFILE;
  }
  std::vector<float> fl(kFloats);
  for (size_t i = 0; i < kFloats; ++i) {
    const uint32_t u = rd32(24 + 4 * i);
    memcpy(&fl[i], &u, 4);
  }
  int32_t cls[NC];
  for (int i = 0; i < NC; ++i) cls[i] = (int32_t)rd32(24 + 4 * kFloats + 4 * i);
  for (size_t i = 0; i < kFloats; ++i)
    if (!std::isfinite(fl[i])) {
      set_error("bfs_selector_load: %s holds a non-finite value at float %zu", path, i);
      return BFS_EFILE;
    }
  const float *p = fl.data(), *mean = p + NPARAM, *stdv = mean + NF, *fmin = stdv + NF, *fmax = fmin + NF;
  const float min_conf = fmax[NF];
  const int rc = bfs_selector_set(p, mean, stdv, fmin, fmax, min_conf, cls);
  return rc == BFS_EINVAL ? BFS_EFILE : rc;
}

int bfs_selector_clear(void) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  g_sel[cur_dev()].loaded = false;
  return BFS_OK;
}

int bfs_selector_loaded(void) { return selector_loaded() ? 1 : 0; }

int bfs_mlp_forward(const float *params, const float *x, int32_t batch, float *logits, void *stream) {
  if (!params || !x || !logits || batch < 0) return BFS_EINVAL;
  if (batch == 0) return BFS_OK;
  int grid = std::min((batch + 3) / 4, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(MLP_BLOCK), 0, (hipStream_t)stream, params, x, batch, logits,
                     (int *)nullptr, (float *)nullptr);
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipStreamSynchronize((hipStream_t)stream));
  return BFS_OK;
}

int bfs_mlp_predict(const float *params, const float *x, int32_t batch, int32_t *cls, float *conf, void *stream) {
  if (!params || !x || !cls || !conf || batch < 0) return BFS_EINVAL;
  if (batch == 0) return BFS_OK;
  int grid = std::min((batch + 3) / 4, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(MLP_BLOCK), 0, (hipStream_t)stream, params, x, batch,
                     (float *)nullptr, cls, conf);
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipStreamSynchronize((hipStream_t)stream));
  return BFS_OK;
}

int bfs_mlp_loss_grad(const float *params, const float *x, const int32_t *labels, int32_t batch, float *grad,
                      float *loss, void *stream) {
  if (!params || !x || !labels || !grad || batch <= 0) return BFS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  BFS_HIP(hipMemsetAsync(grad, 0, NPARAM * sizeof(float), s));
  if (loss) BFS_HIP(hipMemsetAsync(loss, 0, sizeof(float), s));
  int grid = (batch + GRAD_ROWS - 1) / GRAD_ROWS;
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(MLP_BLOCK), 0, s, params, x, labels, batch, grad, loss);
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipStreamSynchronize(s));
  return BFS_OK;
}

int bfs_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, float beta1,
                 float beta2, float eps, void *stream) {
  if (!params || !grad || !m || !v || step <= 0) return BFS_EINVAL;
  float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v,
                     NPARAM, lr, beta1, beta2, eps, c1, c2);
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipStreamSynchronize((hipStream_t)stream));
  return BFS_OK;
}

int bfs_level_features(const bfs_stats *st, int32_t n, int32_t nnz, float *feats) {
  if (!st || !feats || n <= 0 || !st->level_frontier || !st->level_frontier_edges || !st->level_unvisited ||
      !st->level_unvisited_edges || !st->level_frontier_ld || !st->level_frontier_ld2) {
    set_error("bfs_level_features: missing per-level arrays");
    return BFS_EINVAL;
  }
  int L = std::min(st->num_levels, st->level_capacity);
  for (int k = 0; k < L; ++k)
    level_features((double)n, (double)nnz, (double)k, (double)st->level_frontier[k],
                   (double)st->level_frontier_edges[k], (double)st->level_unvisited[k],
                   (double)st->level_unvisited_edges[k], (double)st->level_frontier_ld[k],
                   (double)st->level_frontier_ld2[k], (double)st->graph_ld, (double)st->graph_ld2, feats + k * NF);
  return BFS_OK;
}

}  // extern "C"
