// Persistent batched solve: one launch runs every task of a batch of
// instances (phase-1 segment sweeps, linking solves, rebuilds) from a queue.
//
// Each resident workgroup repeatedly takes the next ticket of a global
// counter and runs that task of the host-ordered task table. A linking solve
// waits until every segment sweep of its instance has finished, a rebuild
// until its instance's linking solve has; the waits are on per-instance
// counters published with agent-scope release and read with agent-scope
// acquire (the eight XCDs keep separate L2 caches, so both sides need the
// agent-scope fences, not only workgroup barriers).
//
// Deadlock freedom: the table is a topological order of the dependencies, and
// a workgroup takes a ticket only while it is running. A task therefore waits
// only on tasks with smaller tickets, which are held by running workgroups or
// finished; the smallest unfinished ticket never waits, so every task
// finishes and every workgroup eventually draws a ticket past the end of the
// table and exits. This holds for any grid size and any occupancy.
#pragma once

#include <algorithm>

#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

namespace persist_detail {

// The queue protocol runs in wave 0 with every lane active and branches only
// on the wave index made scalar by readfirstlane: no branch at the loop's
// ticket, signal or wait depends on the lane. (A `threadIdx.x == 0` region at
// the loop boundary lets the compiler route the other lanes of wave 0 straight
// back to the loop's first barrier, past the ticket fetch that only lane 0
// would run; as one wave executes both paths under exec masks, the other
// lanes then re-enter the loop with the old ticket while lane 0 waits, and the
// workgroup never advances.)

// Polls before a wait gives up (about ten seconds): every wait ends, even if
// a dependency were never signalled.
constexpr int kMaxPolls = 1 << 24;

// Block until *ctr >= target (wave 0 polls; the workgroup then acquires).
// Returns true, uniformly, if the wait gave up.
LQR_DEV bool wait_at_least(const int32_t* ctr, int target, int wave, int* sflag) {
  if (wave == 0) {
    int polls = 0;
    while (__builtin_amdgcn_readfirstlane(
               __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target &&
           polls < kMaxPolls) {
      __builtin_amdgcn_s_sleep(8);
      ++polls;
    }
    *sflag = polls >= kMaxPolls ? 1 : 0;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return __builtin_amdgcn_readfirstlane(*sflag) != 0;
}

}  // namespace persist_detail

// `sync` holds sync_words(ninst) int32 words, zero at launch. The dynamic LDS
// is lds_items bytes for the tasks plus 16 bytes for the ticket broadcast.
template <int MW, int E>
__global__ __launch_bounds__(kThreads) void k_persistent(const InstDesc* descs,
                                                         const TaskItem* tasks, int ntasks,
                                                         int ninst, int32_t* sync,
                                                         unsigned lds_items) {
  using persist_detail::wait_at_least;
  extern __shared__ double smem[];
  int* sticket = reinterpret_cast<int*>(reinterpret_cast<char*>(smem) + lds_items);
  int* sflag = sticket + 1;
  int32_t* done1 = sync + kSyncDone1;
  int32_t* done2 = done1 + ninst;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int one = lane == 0 ? 1 : 0;  // lane 0 counts, the other lanes add zero
  // a workgroup never runs more than ntasks tasks: the bound only guarantees
  // that the loop ends
  for (int iter = 0; iter <= ntasks; ++iter) {
    if (wave == 0) {
      const int v = __hip_atomic_fetch_add(sync + kSyncHead, one, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      *sticket = __builtin_amdgcn_readfirstlane(v);  // lane 0's ticket, same value from every lane
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(*sticket);
    if (t >= ntasks) break;
    const TaskItem w = tasks[t];
    const int inst = __builtin_amdgcn_readfirstlane(w.inst);
    const int phase = __builtin_amdgcn_readfirstlane(w.phase);
    const InstDesc d = descs[inst];
    bool gave_up = false;
    if (phase == 1) {
      phase1_item<MW, E>(d, w.seg, smem);
    } else if (phase == 2) {
      gave_up = wait_at_least(done1 + inst, d.J, wave, sflag);
      couple_item<persist_nw(E != kEngValu), fp64_engine(E)>(d, smem);
    } else {
      gave_up = wait_at_least(done2 + inst, 1, wave, sflag);
      phase3_item<MW, E>(d, w.seg, smem);
    }
    if (gave_up && wave == 0)
      __hip_atomic_store(d.info, LQR_INFO_QUEUE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // publish this task's global writes, then count it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave == 0) {
      if (phase == 1)
        __hip_atomic_fetch_add(done1 + inst, one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      else if (phase == 2)
        __hip_atomic_store(done2 + inst, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Launch the <MW, E> variant with one workgroup per resident slot
// (occupancy x compute units, at most ntasks). `lds` includes the ticket slot.
template <int MW, int E>
hipError_t launch_persistent_variant(const InstDesc* descs, const TaskItem* tasks, int ntasks,
                                     int ninst, int32_t* sync, unsigned lds_items, size_t lds,
                                     int cus, int* grid_out, hipStream_t stream) {
  const void* k = (const void*)&k_persistent<MW, E>;
  hipError_t e = ensure_dynamic_lds(k, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int grid = std::min(ntasks, per_cu * cus);
  if (grid_out) *grid_out = grid;
  hipLaunchKernelGGL((k_persistent<MW, E>), dim3(grid), dim3(kThreads), lds, stream, descs, tasks,
                     ntasks, ninst, sync, lds_items);
  return hipGetLastError();
}

#define LQR_PERSISTENT_DECL(W, M)                                                              \
  extern template hipError_t launch_persistent_variant<W, M>(                                   \
      const InstDesc*, const TaskItem*, int, int, int32_t*, unsigned, size_t, int, int*,        \
      hipStream_t);
#define LQR_PERSISTENT_INST(W, M)                                                              \
  template hipError_t launch_persistent_variant<W, M>(const InstDesc*, const TaskItem*, int, int, \
                                                      int32_t*, unsigned, size_t, int, int*,    \
                                                      hipStream_t);

}  // namespace lqr
