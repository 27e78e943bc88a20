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

hipError_t launch_phase(const InstDesc& d, int phase, size_t lds, int eng, hipStream_t stream) {
  switch (phase) {
    case 1:
      if (d.n <= kSmallMax && d.m <= kSmallMax) return launch_small_phase1(d, stream);
      return launch_k_phase1(d, nullptr, nullptr, d.J, kernel_width(d.m, eng), eng, lds, stream);
    case 2:
      if (use_link_tree(d.n, d.J)) return launch_link_tree(d, lds, stream);
      return launch_k_phase2(d, nullptr, nullptr, 1, d.n, launch_engine(d.n, false), lds, stream);
    case 3:
      if (d.n <= kSmallMax && d.m <= kSmallMax) return launch_small_phase3(d, stream);
      return launch_k_phase3(d, nullptr, nullptr, d.J, kernel_width(d.m, eng), eng, lds, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_parallel(const InstDesc& d, size_t lds1, size_t lds2, size_t lds3, int eng,
                           hipStream_t stream) {
  hipError_t e;
  if ((e = launch_phase(d, 1, lds1, eng, stream)) != hipSuccess) return e;
  if ((e = launch_phase(d, 2, lds2, eng, stream)) != hipSuccess) return e;
  return launch_phase(d, 3, lds3, eng, stream);
}

hipError_t launch_serial(const InstDesc& d, size_t lds, int eng, hipStream_t stream) {
  return launch_k_serial(d, nullptr, nullptr, 1, kernel_width(d.m, eng), eng, lds, stream);
}

hipError_t launch_parallel_batched(const InstDesc* descs, const WorkItem* items, int nitems,
                                   int ninst, int max_n, int max_m, size_t lds1, size_t lds2,
                                   size_t lds3, int eng, hipStream_t stream) {
  const InstDesc none{};
  hipError_t e;
  if ((e = launch_k_phase1(none, descs, items, nitems, kernel_width(max_m, eng), eng, lds1, stream)) !=
      hipSuccess)
    return e;
  if ((e = launch_k_phase2(none, descs, nullptr, ninst, max_n, launch_engine(max_n, false), lds2,
                           stream)) != hipSuccess)
    return e;
  return launch_k_phase3(none, descs, items, nitems, kernel_width(max_m, eng), eng, lds3, stream);
}

hipError_t launch_serial_batched(const InstDesc* descs, int ninst, int max_m, int eng, size_t lds,
                                 hipStream_t stream) {
  const InstDesc none{};
  return launch_k_serial(none, descs, nullptr, ninst, kernel_width(max_m, eng), eng, lds, stream);
}

}  // namespace lqr
