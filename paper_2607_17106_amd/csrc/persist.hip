// Whole-search persistent kernel: one cooperative launch runs every level of
// a single-source BFS (Cascade 1 iterated to convergence) on a grid that is
// fully resident, separating the phases of a level with grid barriers
// instead of kernel boundaries.  Each level: the chosen step body (same code
// as the per-step kernels), a barrier, workgroup 0 reduces the counters and
// decides the next level's variant, a barrier.  This removes the per-level
// host round trip and the per-kernel dispatch gaps, which dominate levels
// whose frontier is small (high-diameter graphs, the tails of R-MAT searches).
//
// Grid barrier: workgroups arrive on one of 64 counters (own 64-byte lines;
// same-address device atomics serialise across XCDs), workgroup 0 sums them
// with one load per lane and releases a flag the others poll.  Release and
// acquire are agent-scope fences, which write back / invalidate the XCD's L2
// so data written before the barrier is seen after it on every XCD.  Every
// wait is bounded: on timeout an error flag is raised and every workgroup
// leaves the kernel.
#include "common.hpp"
#include "step_bodies.hpp"
#include "selector_dev.hpp"
#include "persist.hpp"

namespace bfs {

constexpr long long SPIN_LIMIT = 1ll << 23;

__device__ __forceinline__ u32 ld_acq(const u32 *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 ld_rlx(const u32 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns false (in every thread of the workgroup) if the barrier failed.
__device__ bool grid_sync(GridBar *b, u32 &epoch) {
  __shared__ int s_ok;
  __syncthreads();
  ++epoch;
  if (threadIdx.x < WAVE) {
    bool ok = true;
    if (threadIdx.x == 0) {
      __threadfence();
      atomicAdd(&b->arrive[blockIdx.x & 63].v, 1u);
    }
    if (blockIdx.x == 0) {
      const u32 target = epoch * gridDim.x;
      long long spins = 0;
      for (;;) {
        u32 sum = ld_rlx(&b->arrive[lane()].v);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
        if (sum >= target) break;
        const bool err = __ballot(lane() == 0 && ld_rlx(&b->err.v) != 0u) != 0ull;
        if (err || ++spins > SPIN_LIMIT) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (threadIdx.x == 0) {
        if (!ok) __hip_atomic_store(&b->err.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __hip_atomic_store(&b->flag.v, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else if (threadIdx.x == 0) {
      long long spins = 0;
      while (ld_acq(&b->flag.v) < epoch) {
        if (ld_rlx(&b->err.v) != 0u || ++spins > SPIN_LIMIT) {
          ok = false;
          __hip_atomic_store(&b->err.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __threadfence();
    }
    if (threadIdx.x == 0) s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ void set_level(StepArgs &a, const PersistArgs &P, int k) {
  a.k = k;
  a.fb_cur = P.fb[k % 3];
  a.fb_next = P.fb[(k + 1) % 3];
  a.fb_dead = P.fb[(k + 2) % 3];
  a.q_cur = P.q[k % 2];
  a.q_next = P.q[(k + 1) % 2];
  a.c_cur = &P.ring[k % RING].tot;
  a.seg_cur = P.ring[k % RING].seg;
  a.sh_next = P.ring[(k + 1) % RING].sh;
  a.sh_zero = P.ring[(k + 2) % RING].sh;
}

__global__ __launch_bounds__(BLOCK) void k_bfs_persistent(PersistArgs P) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_dedup[SM_DEDUP / 4];
  u32 epoch = 0;
  StepArgs a = P.base;
  a.gate = -1;
  set_level(a, P, 0);
  body_reset(a, P.src, P.ring);
  if (!grid_sync(P.bar, epoch)) return;
  if (blockIdx.x == 0) {
    body_reset_f0(a, P.src, P.ring);
    __syncthreads();
    __threadfence();
    body_log_f0(P.ring, P.log, P.ctl);
    if (threadIdx.x == 0) P.log[0].t = wall_clock64();
    __syncthreads();
    __threadfence();
    if (P.decide && threadIdx.x < WAVE)
      body_select(P.sd, P.ring, 0, a.n, P.nnz, 1, P.use_net, P.log, smem);
  }
  if (!grid_sync(P.bar, epoch)) return;
  for (int k = 0;; ++k) {
    set_level(a, P, k);
    const u32 cnt = a.c_cur->count;
    if (cnt == 0u) break;
    if (k >= P.maxlev) {
      if (blockIdx.x == 0 && threadIdx.x == 0) P.ctl->pad[0] = 2;  // level cap
      break;
    }
    int dec = P.decide ? a.c_cur->decision : P.sched[min(k, P.sched_len - 1)];
    if (dec < 0 || dec >= BFS_NUM_VARIANTS) dec = P.push_v;
    clear_dead(a);
    bool ok = true;
    switch (dec) {
      case BFS_V_PUSH_Q_THREAD:
        body_push_q_thread<true>(a, smem);
        break;
      case BFS_V_PUSH_Q_BLOCK:
        body_push_q_block<true>(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_push_hubs<true>(a, smem);
        break;
      case BFS_V_PUSH_Q_MERGE:
        body_merge_scan_local(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_merge_scan_chunks(a, smem);
        ok = ok && grid_sync(P.bar, epoch);
        if (ok) body_push_merge<true>(a, smem);
        break;
      case BFS_V_PUSH_B_ATOMIC:
        body_push_b<true>(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_push_hubs<true>(a, smem);
        break;
      case BFS_V_PUSH_B_NOATOMIC:
        body_push_b<false>(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_push_hubs<false>(a, smem);
        ok = ok && grid_sync(P.bar, epoch);
        if (ok) body_noatom_update(a);
        break;
      case BFS_V_PUSH_Q_NOATOMIC:
        body_push_q_block<false>(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_push_hubs<false>(a, smem);
        ok = ok && grid_sync(P.bar, epoch);
        if (ok) body_noatom_update(a);
        break;
      case BFS_V_PULL_VIS:
        body_pull<true>(a);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_merge_vis(a);
        break;
      case BFS_V_PUSH_Q_FILTER: {
        body_merge_scan_local(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_merge_scan_chunks(a, smem);
        ok = ok && grid_sync(P.bar, epoch);
        const int chunks = ok ? (int)(((long long)a.c_cur->total_e + a.tmpcap - 1) / a.tmpcap) : 0;
        for (int r = 0; ok && r < chunks; ++r) {  // uniform: every workgroup read the same total
          body_push_merge<true, true>(a, smem, r);
          ok = grid_sync(P.bar, epoch);
          if (ok) body_filter_tmp(a, r);
          ok = ok && grid_sync(P.bar, epoch);
        }
        break;
      }
      case BFS_V_PUSH_B_FILTER: {
        body_wscan_local(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_merge_scan_chunks(a, smem, true);
        ok = ok && grid_sync(P.bar, epoch);
        const int chunks = ok ? (int)(((long long)a.c_cur->total_e + a.tmpcap - 1) / a.tmpcap) : 0;
        for (int r = 0; ok && r < chunks; ++r) {  // uniform: every workgroup read the same total
          body_adv_tmp_b(a, smem, r);
          ok = grid_sync(P.bar, epoch);
          if (ok) body_filter_tmp(a, r);
          ok = ok && grid_sync(P.bar, epoch);
        }
        break;
      }
      case BFS_V_PUSH_Q_DEDUP:
        body_push_q_block<false, true>(a, smem, s_dedup);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_push_hubs<false, true>(a, smem, s_dedup);
        ok = ok && grid_sync(P.bar, epoch);
        if (ok) body_filter_tmp(a, 0);
        break;
      case BFS_V_PUSH_P3:
        body_push_p3(a, smem);
        ok = grid_sync(P.bar, epoch);
        if (ok) body_push_hubs<false>(a, smem);
        ok = ok && grid_sync(P.bar, epoch);
        if (ok) body_p3_update(a);
        break;
      default:  // BFS_V_PULL_B
        body_pull<false>(a);
        break;
    }
    if (!ok || !grid_sync(P.bar, epoch)) break;
    if (blockIdx.x == 0) {
      body_finish(&P.ring[(k + 1) % RING], a.qcap, k + 1, P.log, P.ctl, smem);
      if (threadIdx.x == 0 && k + 1 < LOGCAP) P.log[k + 1].t = wall_clock64();
      if (P.decide) {
        __syncthreads();
        __threadfence();
        if (threadIdx.x < WAVE)
          body_select(P.sd, P.ring, k + 1, a.n, P.nnz, 0, P.use_net, P.log, smem + SM_FINISH);
      }
    }
    if (!grid_sync(P.bar, epoch)) break;
  }
}

static int g_persist_blocks[64] = {0};

hipError_t launch_persistent(const PersistArgs &P, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int &nb = g_persist_blocks[dev & 63];
  if (nb == 0) {
    int per_cu = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bfs_persistent, BLOCK, SM_MAX);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    nb = std::min(per_cu, PERSIST_BLOCKS_PER_CU) * cus;
  }
  void *args[] = {const_cast<PersistArgs *>(&P)};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_bfs_persistent), dim3(nb), dim3(BLOCK), args,
                                    SM_MAX, s);
}

}  // namespace bfs
