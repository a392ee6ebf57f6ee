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

// Argmax over lanes 0..3 (ties to the lowest index) and the top softmax
// probability, 1 / sum_j exp(l_j - l_max).
__device__ inline void argmax_conf(float logit, int *cls, float *conf) {
  float l0 = __shfl(logit, 0), l1 = __shfl(logit, 1), l2 = __shfl(logit, 2), l3 = __shfl(logit, 3);
  float L[4] = {l0, l1, l2, l3};
  int best = 0;
  for (int j = 1; j < NC; ++j)
    if (L[j] > L[best]) best = j;
  float s = 0.f;
  for (int j = 0; j < NC; ++j) s += expf(L[j] - L[best]);
  *cls = best;
  *conf = 1.f / s;
}

// ------------------------------------------------------ device selection
// Runs after the step that produced F_k: updates the running unvisited
// totals, advances the direction rule, evaluates the network on F_k's
// features and stores the choice in ring[k % RING].decision.
// Run by one whole wave.  smem: SM_SELECT bytes.
// bf16 weights staged in LDS before the forward pass (16-byte copies, all in
// flight at once), instead of one dependent 2-byte global load per product.
constexpr int SEL_W16 = (NPARAM * 2 + 15) / 16;  // 16-byte units; the source buffer extends past them

__device__ __forceinline__ void body_select(const SelDevice &sd, RingSlot *ring, int k, int n, int nnz, int init,
                                            int use_net, LevelLog *log, char *smem, int4 *s_wt = nullptr) {
  float *s_x = reinterpret_cast<float *>(smem), *h0 = s_x + NF, *h1 = h0 + NH, *h2 = h1 + NH;
  int &s_hv = *reinterpret_cast<int *>(h2 + NH);
  LevelCtr *c = &ring[k % RING].tot;
  long long *st = reinterpret_cast<long long *>(sd.state);
  const long long nF = c->count;
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
    float f[NF];
    level_features((double)n, (double)nnz, (double)k, (double)nF, (double)c->edges, (double)st[0], (double)st[1],
                   (double)c->ld, (double)c->ld2, (double)sd.gld, (double)sd.gld2, f);
    for (int i = 0; i < NF; ++i) s_x[i] = f[i];
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
  // range check on raw features, then normalise
  bool out_of_range = false;
  float xn = 0.f;
  if (lane() < NF) {
    float r = s_x[lane()];
    out_of_range = r < sd.norm[2 * NF + lane()] || r > sd.norm[3 * NF + lane()];
    xn = (r - sd.norm[lane()]) / sd.norm[NF + lane()];
  }
  const bool any_oor = __ballot(out_of_range) != 0ull;
  __builtin_amdgcn_wave_barrier();
  if (lane() < NF) s_x[lane()] = xn;
  __builtin_amdgcn_wave_barrier();
  const u16 *w = sd.w;
  if (s_wt) {
    const int4 *src = reinterpret_cast<const int4 *>(sd.w);
    for (int i = lane(); i < SEL_W16; i += WAVE) s_wt[i] = src[i];
    __builtin_amdgcn_wave_barrier();
    w = reinterpret_cast<const u16 *>(s_wt);
  }
  float z1, z2;
  float logit = forward_row(WBf16{w}, sd.p, s_x, h0, h1, h2, z1, z2);
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
