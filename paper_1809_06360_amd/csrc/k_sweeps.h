// Kernels of the segment sweeps: phase 1 (parametric sweep of every segment
// but the last, plain recursion of the last), phase 3 (rebuild from the exact
// boundary values and forward simulation) and the plain serial recursion (the
// GPU baseline). Each is instantiated per register width MW (8..64, the padded
// input dimension m held in registers by the elimination) and per product
// engine E (FP64 vector ALUs, FP64 or FP32 matrix cores; see pgemm_sub), so
// that each launch runs one compact variant. The launchers of one (kernel,
// engine) pair are compiled in a translation unit of their own (k_sweep_*.hip)
// so that the library builds in parallel.
#pragma once

#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

template <int MW, int E>
__global__ __launch_bounds__(kThreads) void k_phase1(InstDesc single, const InstDesc* descs,
                                                     const WorkItem* items) {
  extern __shared__ double smem[];
  InstDesc d;
  int seg;
  select_item(single, descs, items, d, seg);
  phase1_item<MW, E>(d, seg, smem);
}

template <int MW, int E>
__global__ __launch_bounds__(kThreads) void k_phase3(InstDesc single, const InstDesc* descs,
                                                     const WorkItem* items) {
  extern __shared__ double smem[];
  InstDesc d;
  int seg;
  select_item(single, descs, items, d, seg);
  phase3_item<MW, E>(d, seg, smem);
}

template <int MW, int E>
__global__ __launch_bounds__(kThreads) void k_serial(InstDesc single, const InstDesc* descs,
                                                     const WorkItem* items) {
  extern __shared__ double smem[];
  InstDesc d;
  int seg;
  select_item(single, descs, items, d, seg);
  serial_item<MW, E>(d, smem);
}

// Which sweep kernel a launcher runs.
constexpr int kSweepSerial = 0, kSweepPhase1 = 1, kSweepPhase3 = 3;

template <int KIND, int MW, int E>
const void* sweep_kernel() {
  if constexpr (KIND == kSweepPhase1) return (const void*)&k_phase1<MW, E>;
  else if constexpr (KIND == kSweepPhase3) return (const void*)&k_phase3<MW, E>;
  else return (const void*)&k_serial<MW, E>;
}

template <int KIND, int MW, int E>
hipError_t launch_sweep_variant(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                                unsigned grid, size_t lds, hipStream_t stream) {
  const void* k = sweep_kernel<KIND, MW, E>();
  hipError_t e = ensure_dynamic_lds(k, lds);
  if (e != hipSuccess) return e;
  if constexpr (KIND == kSweepPhase1)
    hipLaunchKernelGGL((k_phase1<MW, E>), dim3(grid), dim3(kThreads), lds, stream, single, descs, items);
  else if constexpr (KIND == kSweepPhase3)
    hipLaunchKernelGGL((k_phase3<MW, E>), dim3(grid), dim3(kThreads), lds, stream, single, descs, items);
  else
    hipLaunchKernelGGL((k_serial<MW, E>), dim3(grid), dim3(kThreads), lds, stream, single, descs, items);
  return hipGetLastError();
}

// Launch the KIND kernel of engine E at register width pad_rows(width).
// Width 8 exists only for the vector-ALU engine (see with_variant).
template <int KIND, int E>
hipError_t launch_sweep(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                        unsigned grid, int width, size_t lds, hipStream_t stream) {
  switch (pad_rows(width)) {
    case 8:
      if constexpr (E == 0)
        return launch_sweep_variant<KIND, 8, E>(single, descs, items, grid, lds, stream);
      else
        return hipErrorInvalidValue;
    case 16: return launch_sweep_variant<KIND, 16, E>(single, descs, items, grid, lds, stream);
    case 24: return launch_sweep_variant<KIND, 24, E>(single, descs, items, grid, lds, stream);
    case 32: return launch_sweep_variant<KIND, 32, E>(single, descs, items, grid, lds, stream);
    case 48: return launch_sweep_variant<KIND, 48, E>(single, descs, items, grid, lds, stream);
    case 64: return launch_sweep_variant<KIND, 64, E>(single, descs, items, grid, lds, stream);
  }
  return hipErrorInvalidValue;
}

#define LQR_SWEEP_LAUNCH_ARGS                                                                 \
  const InstDesc&, const InstDesc*, const WorkItem*, unsigned, int, size_t, hipStream_t
#define LQR_SWEEP_DECL(KIND, E) extern template hipError_t launch_sweep<KIND, E>(LQR_SWEEP_LAUNCH_ARGS);
#define LQR_SWEEP_INST(KIND, E) template hipError_t launch_sweep<KIND, E>(LQR_SWEEP_LAUNCH_ARGS);

}  // namespace lqr
