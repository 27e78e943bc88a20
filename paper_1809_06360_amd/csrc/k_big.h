// Kernels of the large-state path's segment sweeps (big_device.h): phase 1,
// phase 3 and the plain serial recursion, one 256-thread workgroup per segment
// (per instance for the serial kernel), instantiated per product engine in
// k_big_e1.hip (FP64) and k_big_e2.hip (FP32 matrix cores).
#pragma once

#include "big_device.h"
#include "lqr_launch.h"

namespace lqr {

template <int E>
__global__ __launch_bounds__(big::kSweepThreads) void k_big_phase1(InstDesc d) {
  extern __shared__ double smem[];
  big::phase1_item<E>(d, blockIdx.x, smem);
}

template <int E>
__global__ __launch_bounds__(big::kSweepThreads) void k_big_phase3(InstDesc d) {
  extern __shared__ double smem[];
  big::phase3_item<E>(d, blockIdx.x, smem);
}

template <int E>
__global__ __launch_bounds__(big::kSweepThreads) void k_big_serial(InstDesc d) {
  extern __shared__ double smem[];
  big::serial_item<E>(d, smem);
}

// kind 1: phase 1, kind 3: phase 3 (J workgroups); kind 0: serial (one).
template <int E>
hipError_t launch_big_sweep_e(const InstDesc& d, int kind, size_t lds, hipStream_t stream) {
  const void* k = kind == 1   ? (const void*)&k_big_phase1<E>
                  : kind == 3 ? (const void*)&k_big_phase3<E>
                              : (const void*)&k_big_serial<E>;
  hipError_t e = ensure_dynamic_lds(k, lds);
  if (e != hipSuccess) return e;
  if (kind == 1)
    hipLaunchKernelGGL(k_big_phase1<E>, dim3(d.J), dim3(big::kSweepThreads), lds, stream, d);
  else if (kind == 3)
    hipLaunchKernelGGL(k_big_phase3<E>, dim3(d.J), dim3(big::kSweepThreads), lds, stream, d);
  else
    hipLaunchKernelGGL(k_big_serial<E>, dim3(1), dim3(big::kSweepThreads), lds, stream, d);
  return hipGetLastError();
}

extern template hipError_t launch_big_sweep_e<1>(const InstDesc&, int, size_t, hipStream_t);
extern template hipError_t launch_big_sweep_e<2>(const InstDesc&, int, size_t, hipStream_t);

}  // namespace lqr
