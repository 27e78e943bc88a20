// Phase 2: linking solve over the segment boundaries.
#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

// Instantiated per register width MW (8..64, the padded state dimension n held in
// registers by the elimination) and per product engine E (FP64 vector ALUs,
// FP64 or FP32 matrix cores; see pgemm_sub), so that each launch runs one
// compact variant.
template <int MW, int E>
__global__ __launch_bounds__(kThreads) void k_phase2(InstDesc single, const InstDesc* descs,
                                                     const WorkItem* items) {
  extern __shared__ double smem[];
  InstDesc d;
  int seg;
  select_item(single, descs, items, d, seg);
  couple_item<MW, E>(d, smem);
}

template <int W, int M>
struct k_phase2_ref {
  static auto fn() { return &k_phase2<W, M>; }
};

hipError_t launch_k_phase2(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                   unsigned grid, int width, int eng, size_t lds, hipStream_t stream) {
  if (eng != launch_engine(width, false)) return hipErrorInvalidValue;
  return with_link_variant<k_phase2_ref>(width, [&](auto k) -> hipError_t {
    hipError_t e = ensure_dynamic_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, stream, single, descs, items);
    return hipGetLastError();
  });
}

}  // namespace lqr
