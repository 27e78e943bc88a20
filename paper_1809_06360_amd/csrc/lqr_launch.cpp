// Launch sequences of the solver (host code).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "lqr_kernels.h"
#include "lqr_launch.h"

namespace lqr {

hipError_t ensure_dynamic_lds(const void* kernel, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  size_t& have = done[{dev, kernel}];
  if (have >= lds) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) have = lds;
  return e;
}

static bool use_mfma(int n) { return n >= kMfmaMinN; }

hipError_t launch_phase(const InstDesc& d, int phase, size_t lds, hipStream_t stream) {
  const bool mf = use_mfma(d.n);
  switch (phase) {
    case 1: return launch_k_phase1(d, nullptr, nullptr, d.J, d.m, mf, lds, stream);
    case 2: return launch_k_phase2(d, nullptr, nullptr, 1, d.n, mf, lds, stream);
    case 3: return launch_k_phase3(d, nullptr, nullptr, d.J, d.m, mf, lds, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_parallel(const InstDesc& d, size_t lds1, size_t lds2, size_t lds3,
                           hipStream_t stream) {
  hipError_t e;
  if ((e = launch_phase(d, 1, lds1, stream)) != hipSuccess) return e;
  if ((e = launch_phase(d, 2, lds2, stream)) != hipSuccess) return e;
  return launch_phase(d, 3, lds3, stream);
}

hipError_t launch_serial(const InstDesc& d, size_t lds, hipStream_t stream) {
  return launch_k_serial(d, nullptr, nullptr, 1, d.m, use_mfma(d.n), lds, stream);
}

hipError_t launch_parallel_batched(const InstDesc* descs, const WorkItem* items, int nitems,
                                   int ninst, int max_n, int max_m, size_t lds1, size_t lds2,
                                   size_t lds3, hipStream_t stream) {
  const bool mf = use_mfma(max_n);
  const InstDesc none{};
  hipError_t e;
  if ((e = launch_k_phase1(none, descs, items, nitems, max_m, mf, lds1, stream)) != hipSuccess) return e;
  if ((e = launch_k_phase2(none, descs, nullptr, ninst, max_n, mf, lds2, stream)) != hipSuccess) return e;
  return launch_k_phase3(none, descs, items, nitems, max_m, mf, lds3, stream);
}

hipError_t launch_serial_batched(const InstDesc* descs, int ninst, int max_n, int max_m, size_t lds,
                                 hipStream_t stream) {
  const InstDesc none{};
  return launch_k_serial(none, descs, nullptr, ninst, max_m, use_mfma(max_n), lds, stream);
}

}  // namespace lqr
