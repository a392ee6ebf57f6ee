// Device side of the per-level variant choice: bf16 helpers, the selector
// network's forward pass and the selection body (direction rule + network),
// shared by the per-level kernel (mlp.hip) and the persistent search kernel.
//
// Network: x (12 normalised features) -> h0 = bf16(x)
//   z1 = b1 + W1 h0, h1 = bf16(relu(z1))
//   z2 = b2 + W2 h1, h2 = bf16(relu(z2))
//   logits = b3 + W3 h2
// with W = bf16(W_master).  Each output is accumulated in fp32 starting from
// its bias, adding products in ascending input order.  A product of two bf16
// values is exact in fp32, so a fused multiply-add gives the same result as a
// separate multiply and add; the order is what makes the result reproducible.
#pragma once
#include "common.hpp"
#include "selector.hpp"

namespace bfs {

constexpr int SM_SELECT = (NF + 3 * NH + 1) * 4;

// fp32 -> bf16 bits, round to nearest even (NaN kept quiet).
__host__ __device__ inline u16 f2bf(float f) {
  union { float f; u32 u; } x;
  x.f = f;
  if ((x.u & 0x7f800000u) == 0x7f800000u && (x.u & 0x007fffffu)) return (u16)((x.u >> 16) | 0x40u);
  u32 lsb = (x.u >> 16) & 1u;
  return (u16)((x.u + 0x7fffu + lsb) >> 16);
}
__host__ __device__ inline float bf2f(u16 b) {
  union { float f; u32 u; } x;
  x.u = ((u32)b) << 16;
  return x.f;
}
__device__ inline float bfr(float f) { return bf2f(f2bf(f)); }

// Weight access: pre-rounded bf16 storage (selector) or fp32 masters rounded
// on the fly (training); both yield the same fp32 values.
struct WBf16 {
  const u16 *w;
  __device__ float operator()(int i) const { return bf2f(w[i]); }
};
struct WMaster {
  const float *p;
  __device__ float operator()(int i) const { return bfr(p[i]); }
};

// Forward of one row by one wave (64 lanes).  h0/h1/h2 are wave-private LDS
// rows; returns logits in lanes 0..3 (other lanes return 0) and leaves the
// pre-activations z1/z2 in the caller's registers.
template <class W>
__device__ inline float forward_row(const W &wt, const float *p, const float *x, float *h0, float *h1, float *h2,
                                    float &z1, float &z2) {
  const int l = lane();
  if (l < NF) h0[l] = bfr(x[l]);
  __builtin_amdgcn_wave_barrier();
  float acc = p[OFF_B1 + l];
  for (int k = 0; k < NF; ++k) acc = acc + h0[k] * wt(OFF_W1 + l * NF + k);
  z1 = acc;
  h1[l] = bfr(fmaxf(acc, 0.f));
  __builtin_amdgcn_wave_barrier();
  acc = p[OFF_B2 + l];
  for (int k = 0; k < NH; ++k) acc = acc + h1[k] * wt(OFF_W2 + l * NH + k);
  z2 = acc;
  h2[l] = bfr(fmaxf(acc, 0.f));
  __builtin_amdgcn_wave_barrier();
  float out = 0.f;
  if (l < NC) {
    acc = p[OFF_B3 + l];
    for (int k = 0; k < NH; ++k) acc = acc + h2[k] * wt(OFF_W3 + l * NH + k);
    out = acc;
  }
  return out;
}

// One lane's rows of the network, kept in registers by the wave that
// evaluates it: lane l holds W1[l][*] and W2[l][*] (bf16 pairs as stored) and
// its two biases; lanes 0..3 also W3[l][*] and b3[l].  The per-level kernel
// loads them at its start, so the loads overlap its counter reduction, and
// the forward pass then reads only the layer inputs (LDS broadcasts) -- not
// two LDS words per product as a staged copy of the matrices would.
struct NetRegs {
  u32 w1[NF / 2], w2[NH / 2], w3[NH / 2];
  float b1, b2, b3;
};

// Loads lane l's rows (one wave).  Byte offsets of the rows: W1 24 l,
// W2 1664 + 128 l, W3 9984 + 128 l in a 256-byte aligned buffer, so the
// 8- and 16-byte loads are aligned.
__device__ __forceinline__ void load_net(const SelDevice &sd, NetRegs &r) {
  const int l = lane();
  const uint2 *p1 = reinterpret_cast<const uint2 *>(sd.w + OFF_W1 + l * NF);
#pragma unroll
  for (int i = 0; i < NF / 4; ++i) {
    const uint2 x = p1[i];
    r.w1[2 * i] = x.x;
    r.w1[2 * i + 1] = x.y;
  }
  const uint4 *p2 = reinterpret_cast<const uint4 *>(sd.w + OFF_W2 + l * NH);
#pragma unroll
  for (int i = 0; i < NH / 8; ++i) {
    const uint4 x = p2[i];
    r.w2[4 * i] = x.x;
    r.w2[4 * i + 1] = x.y;
    r.w2[4 * i + 2] = x.z;
    r.w2[4 * i + 3] = x.w;
  }
  r.b1 = sd.p[OFF_B1 + l];
  r.b2 = sd.p[OFF_B2 + l];
  r.b3 = 0.f;
#pragma unroll
  for (int i = 0; i < NH / 2; ++i) r.w3[i] = 0u;
  if (l < NC) {
    const uint4 *p3 = reinterpret_cast<const uint4 *>(sd.w + OFF_W3 + l * NH);
#pragma unroll
    for (int i = 0; i < NH / 8; ++i) {
      const uint4 x = p3[i];
      r.w3[4 * i] = x.x;
      r.w3[4 * i + 1] = x.y;
      r.w3[4 * i + 2] = x.z;
      r.w3[4 * i + 3] = x.w;
    }
    r.b3 = sd.p[OFF_B3 + l];
  }
}

// Element k of a row of bf16 pairs (little-endian: the even element is the
// low half).
__device__ __forceinline__ float bf_at(const u32 *row, int k) {
  const u32 u = row[k >> 1];
  union { u32 u; float f; } x;
  x.u = (k & 1) ? (u & 0xffff0000u) : (u << 16);
  return x.f;
}

// forward_row from register rows: the same values, the same order of
// accumulation (from the bias, ascending input), so the same logits.
__device__ __forceinline__ float forward_row_regs(const NetRegs &r, const float *x, float *h0, float *h1, float *h2) {
  const int l = lane();
  if (l < NF) h0[l] = bfr(x[l]);
  __builtin_amdgcn_wave_barrier();
  float acc = r.b1;
#pragma unroll
  for (int k = 0; k < NF; ++k) acc = acc + h0[k] * bf_at(r.w1, k);
  h1[l] = bfr(fmaxf(acc, 0.f));
  __builtin_amdgcn_wave_barrier();
  acc = r.b2;
#pragma unroll
  for (int k = 0; k < NH; ++k) acc = acc + h1[k] * bf_at(r.w2, k);
  h2[l] = bfr(fmaxf(acc, 0.f));
  __builtin_amdgcn_wave_barrier();
  acc = r.b3;
#pragma unroll
  for (int k = 0; k < NH; ++k) acc = acc + h2[k] * bf_at(r.w3, k);
  return l < NC ? acc : 0.f;
}

// Argmax over lanes 0..3 (ties to the lowest index) and the top softmax
// probability, 1 / sum_j exp(l_j - l_max).
__device__ inline void argmax_conf(float logit, int *cls, float *conf) {
  static_assert(NC == 4, "four classes");
  const float l0 = lane_bcast(logit, 0), l1 = lane_bcast(logit, 1), l2 = lane_bcast(logit, 2), l3 = lane_bcast(logit, 3);
  int best = 0;
  float mx = l0;
  if (l1 > mx) { best = 1; mx = l1; }
  if (l2 > mx) { best = 2; mx = l2; }
  if (l3 > mx) { best = 3; mx = l3; }
  float s = 0.f;
  s += expf(l0 - mx);
  s += expf(l1 - mx);
  s += expf(l2 - mx);
  s += expf(l3 - mx);
  *cls = best;
  *conf = 1.f / s;
}

// ------------------------------------------------------ device selection
// Runs after the step that produced F_k: updates the running unvisited
// totals, advances the direction rule, evaluates the network on F_k's
// features and stores the choice in ring[k % RING].decision.
// Run by one whole wave.  smem: SM_SELECT bytes.  REGS: the network is
// evaluated from this lane's rows loaded by load_net (regs), else from the
// weights in global memory.
template <bool REGS = false>
__device__ __forceinline__ void body_select(const SelDevice &sd, RingSlot *ring, int k, int n, int nnz, int init,
                                            int use_net, LevelLog *log, char *smem, const NetRegs &regs = NetRegs{}) {
  float *s_x = reinterpret_cast<float *>(smem), *h0 = s_x + NF, *h1 = h0 + NH, *h2 = h1 + NH;
  int &s_hv = *reinterpret_cast<int *>(h2 + NH);
  LevelCtr *c = &ring[k % RING].tot;
  long long *st = reinterpret_cast<long long *>(sd.state);
  const long long nF = c->count;
  long long nU0 = 0, eU0 = 0;  // lane 0: the unvisited totals after F_k
  if (lane() == 0) {
    if (init) {
      st[0] = (long long)n;
      st[1] = (long long)nnz;
      st[2] = 0;
      st[3] = -1;
    }
    st[0] -= nF;
    st[1] -= (long long)c->in_edges;
    // direction rule
    long long eF = (long long)c->edges, eU = st[1];
    int dir = (int)st[2];
    if (dir == 0) {
      if (eF * HeuristicState::kAlpha > eU) dir = 1;
    } else {
      bool shrinking = st[3] >= 0 && nF < st[3];
      if (nF * HeuristicState::kBeta < (long long)n && shrinking) dir = 0;
    }
    st[2] = dir;
    st[3] = nF;
    s_hv = dir ? sd.pull_v : sd.push_v;
    nU0 = st[0];
    eU0 = st[1];
  }
  __builtin_amdgcn_wave_barrier();
  if (!use_net) {  // direction rule only
    if (lane() == 0) {
      c->decision = s_hv;
      c->fallback = 0;
      if (log && k < LOGCAP) {
        log[k].variant = s_hv;
        log[k].fallback = 0;
      }
    }
    return;
  }
  // the level's raw features, one per lane (the unvisited totals st[0..1]
  // were updated by lane 0 above); range check, then normalise
  bool out_of_range = false;
  float xn = 0.f;
  const long long nU = (long long)lane_bcast((u64)nU0, 0);
  const long long eU = (long long)lane_bcast((u64)eU0, 0);
  if (lane() < NF) {
    const float r = level_feature(lane(), (double)n, (double)nnz, (double)k, (double)nF, (double)c->edges,
                                  (double)nU, (double)eU, (double)c->ld, (double)c->ld2, (double)sd.gld,
                                  (double)sd.gld2);
    out_of_range = r < sd.norm[2 * NF + lane()] || r > sd.norm[3 * NF + lane()];
    xn = (r - sd.norm[lane()]) / sd.norm[NF + lane()];
  }
  const bool any_oor = __ballot(out_of_range) != 0ull;
  __builtin_amdgcn_wave_barrier();
  if (lane() < NF) s_x[lane()] = xn;
  __builtin_amdgcn_wave_barrier();
  float logit;
  if (REGS) {
    logit = forward_row_regs(regs, s_x, h0, h1, h2);
  } else {
    float z1, z2;
    logit = forward_row(WBf16{sd.w}, sd.p, s_x, h0, h1, h2, z1, z2);
  }
  int cls;
  float conf;
  argmax_conf(logit, &cls, &conf);
  if (lane() == 0) {
    int fb = any_oor || !(conf >= sd.min_conf);
    c->decision = fb ? s_hv : sd.cls[cls];
    c->fallback = fb;
    if (log && k < LOGCAP) {
      log[k].variant = c->decision;
      log[k].fallback = fb;
    }
  }
}

}  // namespace bfs
