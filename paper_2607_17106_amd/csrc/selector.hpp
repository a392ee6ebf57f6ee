// Per-level variant choice: Beamer's direction rule and the learned selector
// network (12 -> 64 -> 64 -> 4, bf16 weights, fp32 accumulation).
#pragma once
#include "common.hpp"

namespace bfs {

typedef unsigned short u16;

// Beamer, Asanovic, Patterson, "Direction-Optimizing Breadth-First Search"
// (SC 2012): alpha = 14, beta = 24.
struct HeuristicState {
  static constexpr long long kAlpha = 14, kBeta = 24;
  int dir = 0;             // 0 top-down (push), 1 bottom-up (pull)
  long long prev_nf = -1;
  void step(long long n, long long nF, long long eF, long long eU);
};

constexpr int NF = BFS_MLP_NFEAT, NH = 64, NC = BFS_MLP_NCLASS;
constexpr int OFF_W1 = 0, OFF_B1 = 768, OFF_W2 = 832, OFF_B2 = 4928, OFF_W3 = 4992, OFF_B3 = 5248;
constexpr int NPARAM = BFS_MLP_NPARAM;

// Raw feature i of one level (see bfs_eeds.h).  Evaluated in fp64 and
// rounded to fp32, on the host (trainer) and on the device (selector) alike;
// the device computes the 12 on 12 lanes at once.  Every feature is either
// log2(1 + a) or a / b - (c / b)^2 (c = 0 for a plain ratio, which leaves
// a / b unchanged), so the lanes pick their operands and then all run the
// same two operations -- one log2 and one division path instead of a
// branch per feature, which a wave would run one after another.
__host__ __device__ inline float level_feature(int i, double n, double nnz, double k, double nF, double eF, double nU,
                                               double eU, double fld, double fld2, double gld, double gld2) {
  double a = 0.0, b = 1.0, c = 0.0;
  bool lg = false;
  switch (i) {
    case 0: lg = true; a = nF; break;
    case 1: lg = true; a = eF; break;
    case 2: lg = true; a = nU; break;
    case 3: lg = true; a = eU; break;
    case 4: a = nF; b = n; break;
    case 5: if (nnz > 0) { a = eF; b = nnz; } break;
    case 6: a = nU; b = n; break;
    case 7: if (nF > 0) { a = fld; b = nF; } break;
    case 8: if (nF > 0) { a = fld2; b = nF; c = fld; } break;  // variance: E[ld^2] - E[ld]^2
    case 9: a = gld; b = n; break;
    case 10: a = gld2; b = n; c = gld; break;
    default: lg = true; a = k; break;
  }
  const double lv = log2(1.0 + a);
  const double m = c / b;
  const double rv = a / b - m * m;
  return (float)(lg ? lv : rv);
}

// All 12 raw features of one level.
__host__ __device__ inline void level_features(double n, double nnz, double k, double nF, double eF, double nU,
                                               double eU, double fld, double fld2, double gld, double gld2,
                                               float *out) {
  for (int i = 0; i < NF; ++i) out[i] = level_feature(i, n, nnz, k, nF, eF, nU, eU, fld, fld2, gld, gld2);
}

// Device-resident selector parameters (set by bfs_selector_set).
struct SelDevice {
  const u16 *w;          // bf16 weights in the flat layout (biases slots unused)
  const float *p;        // fp32 flat parameters (biases read from here)
  const float *norm;     // mean[12], std[12], min[12], max[12]
  float min_conf;
  int cls[NC];
  u64 *state;            // nU, eU, dir, prev_nf (per workspace)
  int push_v, pull_v;
  bool use_net;          // weights present
  u64 gld, gld2;         // graph-wide sums of floor(log2(1 + outdeg)) and its square
};

bool selector_loaded();
SelDevice selector_device(const Workspace &w, int push_v, int pull_v);
// Decides the variant for level k (after F_k's counters are final): the
// network when use_net and weights are loaded, else the direction rule.
hipError_t launch_select(const SelDevice &sd, RingSlot *ring, int k, int n, int nnz, hipStream_t s, bool init,
                         bool use_net, LevelLog *log);
// Level 0 of the host loop (after k_reset alone): F_0 = {src}, its log entry
// and loop control, the choice for level 0 (select), posted to host memory.
hipError_t launch_start_select(const int *rp, const int *cp, int src, RingSlot *slot0, LevelLog *log, LoopCtl *ctl,
                               const SelDevice &sd, int n, int nnz, bool select, bool use_net, LevelCtr *host,
                               u64 *host_seq, u64 seq, hipStream_t s);
// Level-k counter reduction and (select) the choice for level k in one
// launch; with host / host_seq the totals are posted to pinned memory.
hipError_t launch_finish_select(RingSlot *slot, int qcap, int k, LevelLog *log, LoopCtl *ctl, const SelDevice &sd,
                                RingSlot *ring, int n, int nnz, bool select, bool use_net, LevelCtr *host,
                                u64 *host_seq, u64 seq, hipStream_t s);

}  // namespace bfs
