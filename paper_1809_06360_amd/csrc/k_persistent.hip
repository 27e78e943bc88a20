// Persistent batched solve: counter reset and variant dispatch (the kernel
// and its per-width instantiations are in k_persistent.h, k_persistent_w*.hip).
#include "k_persistent.h"

namespace lqr {

#define LQR_DECL2(W) LQR_PERSISTENT_DECL(W, 0) LQR_PERSISTENT_DECL(W, 1) LQR_PERSISTENT_DECL(W, 2)
LQR_PERSISTENT_DECL(8, 0)
LQR_DECL2(16) LQR_DECL2(24) LQR_DECL2(32) LQR_DECL2(48) LQR_DECL2(64)
#undef LQR_DECL2

// Zero the synchronisation words (a kernel, not a memset, so that the launch
// sequence can be captured into a graph and replayed).
__global__ __launch_bounds__(kThreads) void k_clear_sync(int32_t* sync, int words) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < words; i += gridDim.x * kThreads)
    sync[i] = 0;
}

namespace {

int device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
    return 1;
  return v;
}

}  // namespace

hipError_t launch_persistent(const InstDesc* descs, const TaskItem* tasks, int ntasks, int ninst,
                             int32_t* sync, int max_m, int eng, size_t lds_items,
                             int* grid_out, hipStream_t stream) {
  const int words = (int)sync_words(ninst);
  const int cblocks = std::min(64, (words + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_clear_sync, dim3(cblocks), dim3(kThreads), 0, stream, sync, words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  lds_items = (lds_items + 15) / 16 * 16;  // the ticket slot is int-aligned
  const size_t lds = lds_items + 16;
  const int cus = device_cus();
  const unsigned li = (unsigned)lds_items;
  switch (pad_rows(max_m)) {
    case 8:  // vector-ALU engine only (see with_variant)
      if (eng != 0) return hipErrorInvalidValue;
      return launch_persistent_variant<8, 0>(descs, tasks, ntasks, ninst, sync, li, lds, cus,
                                             grid_out, stream);
#define LQR_CASE(W)                                                                            \
  case W:                                                                                      \
    return eng == 2   ? launch_persistent_variant<W, 2>(descs, tasks, ntasks, ninst, sync, li, lds, \
                                                        cus, grid_out, stream)                    \
           : eng == 1 ? launch_persistent_variant<W, 1>(descs, tasks, ntasks, ninst, sync, li, lds, \
                                                        cus, grid_out, stream)                    \
                      : launch_persistent_variant<W, 0>(descs, tasks, ntasks, ninst, sync, li, lds, \
                                                        cus, grid_out, stream);
    LQR_CASE(16) LQR_CASE(24) LQR_CASE(32) LQR_CASE(48) LQR_CASE(64)
#undef LQR_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace lqr
