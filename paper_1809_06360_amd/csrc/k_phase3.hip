// Phase 3: rebuild of gains and value functions from the exact boundary
// values, and forward simulation of every segment.
#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

// Instantiated per register width MW (8..64, the padded input dimension m held in
// registers by the elimination) and per product engine E (FP64 vector ALUs,
// FP64 or FP32 matrix cores; see pgemm_sub), so that each launch runs one
// compact variant.
template <int MW, int E>
__global__ __launch_bounds__(kThreads) void k_phase3(InstDesc single, const InstDesc* descs,
                                                     const WorkItem* items) {
  extern __shared__ double smem[];
  InstDesc d;
  int seg;
  select_item(single, descs, items, d, seg);
  phase3_item<MW, E>(d, seg, smem);
}

template <int W, int M>
struct k_phase3_ref {
  static auto fn() { return &k_phase3<W, M>; }
};

hipError_t launch_k_phase3(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                   unsigned grid, int width, int eng, size_t lds, hipStream_t stream) {
  return with_variant<k_phase3_ref>(width, eng, [&](auto k) -> hipError_t {
    hipError_t e = ensure_dynamic_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, stream, single, descs, items);
    return hipGetLastError();
  });
}

}  // namespace lqr
