// Arguments and launcher of the whole-search persistent kernel (persist.hip).
#pragma once
#include "common.hpp"
#include "selector.hpp"

namespace bfs {

struct alignas(64) BarLine {
  u32 v;
  u32 pad[15];
};
struct GridBar {
  BarLine arrive[64];  // arrival counters, workgroup b uses line b % 64
  BarLine flag;        // epoch released by workgroup 0
  BarLine err;         // set when a wait timed out
};

constexpr int PERSIST_BLOCKS_PER_CU = 2;

struct PersistArgs {
  StepArgs base;        // graph, outputs, visited bitmap, scan/bsum/hubs, qcap, hub
  u64 *fb[3];
  int *q[2];
  RingSlot *ring;
  LevelLog *log;
  LoopCtl *ctl;         // ctl->pad[0]: 2 when the level cap was hit
  u64 *gsum;
  GridBar *bar;
  const int *sched;     // device: variant per level when the host decides
  int sched_len;
  int decide;           // 1: the device chooses each level's variant
  int use_net;          // the selector network decides (else the direction rule)
  int maxlev;
  int src;
  int nnz;
  int push_v;           // fallback for an invalid decision
  SelDevice sd;
};

hipError_t launch_persistent(const PersistArgs &P, hipStream_t s);

}  // namespace bfs
