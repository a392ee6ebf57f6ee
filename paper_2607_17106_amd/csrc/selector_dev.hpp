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

// Selector parameters staged in LDS as fp32 for the per-level kernels: each
// weight matrix transposed (input k of every output adjacent, at [k][out]),
// so the forward pass's lanes read consecutive words.  Read in place, a lane's
// own row lies 128 bytes from the next lane's and all 64 lanes hit one LDS
// bank on every product.
struct SelLds {
  float w1t[NF * NH], w2t[NH * NH], w3t[NH * NC], b1[NH], b2[NH], b3[NC];
};

// Stages the parameters with the NT threads of the workgroup, every global
// load issued before the first LDS store; a __syncthreads() must follow.
template <int NT>
__device__ inline void stage_selector(const SelDevice &sd, SelLds *L) {
  static_assert(NF * NH % NT == 0 && NH * NH % NT == 0 && NH * NC % NT == 0 && NT >= NH, "whole rounds");
  constexpr int N1 = NF * NH / NT, N2 = NH * NH / NT, N3 = NH * NC / NT;
  const int t = threadIdx.x;
  float v1[N1], v2[N2], v3[N3], b1 = 0.f, b2 = 0.f, b3 = 0.f;
#pragma unroll
  for (int j = 0; j < N1; ++j) {  // w1t[k][l] = W1[l][k]
    const int i = t + j * NT;
    v1[j] = bf2f(sd.w[OFF_W1 + (i % NH) * NF + i / NH]);
  }
#pragma unroll
  for (int j = 0; j < N2; ++j) {
    const int i = t + j * NT;
    v2[j] = bf2f(sd.w[OFF_W2 + (i % NH) * NH + i / NH]);
  }
#pragma unroll
  for (int j = 0; j < N3; ++j) {
    const int i = t + j * NT;
    v3[j] = bf2f(sd.w[OFF_W3 + (i % NC) * NH + i / NC]);
  }
  if (t < NH) {
    b1 = sd.p[OFF_B1 + t];
    b2 = sd.p[OFF_B2 + t];
  }
  if (t < NC) b3 = sd.p[OFF_B3 + t];
#pragma unroll
  for (int j = 0; j < N1; ++j) L->w1t[t + j * NT] = v1[j];
#pragma unroll
  for (int j = 0; j < N2; ++j) L->w2t[t + j * NT] = v2[j];
#pragma unroll
  for (int j = 0; j < N3; ++j) L->w3t[t + j * NT] = v3[j];
  if (t < NH) {
    L->b1[t] = b1;
    L->b2[t] = b2;
  }
  if (t < NC) L->b3[t] = b3;
}

// forward_row from the staged parameters: the same values, the same order of
// accumulation, so the same logits.
__device__ inline float forward_row_lds(const SelLds &L, const float *x, float *h0, float *h1, float *h2) {
  const int l = lane();
  if (l < NF) h0[l] = bfr(x[l]);
  __builtin_amdgcn_wave_barrier();
  float acc = L.b1[l];
  for (int k = 0; k < NF; ++k) acc = acc + h0[k] * L.w1t[k * NH + l];
  h1[l] = bfr(fmaxf(acc, 0.f));
  __builtin_amdgcn_wave_barrier();
  acc = L.b2[l];
#pragma unroll 8
  for (int k = 0; k < NH; ++k) acc = acc + h1[k] * L.w2t[k * NH + l];
  h2[l] = bfr(fmaxf(acc, 0.f));
  __builtin_amdgcn_wave_barrier();
  float out = 0.f;
  if (l < NC) {
    acc = L.b3[l];
    for (int k = 0; k < NH; ++k) acc = acc + h2[k] * L.w3t[k * NC + l];
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
// Run by one whole wave.  smem: SM_SELECT bytes.  lds: the parameters staged
// by stage_selector (else read from global memory).
__device__ __forceinline__ void body_select(const SelDevice &sd, RingSlot *ring, int k, int n, int nnz, int init,
                                            int use_net, LevelLog *log, char *smem, const SelLds *lds = nullptr) {
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
  float logit;
  if (lds) {
    logit = forward_row_lds(*lds, s_x, h0, h1, h2);
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
