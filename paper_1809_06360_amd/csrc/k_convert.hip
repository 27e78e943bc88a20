// Conversions between the caller's FP32 arrays and the FP64 staging area of
// the FP32 precision mode (HBM-bound element-wise copies).
#include <hip/hip_runtime.h>

#include "lqr_launch.h"

namespace lqr {

namespace {

constexpr int kCvtThreads = 256;
constexpr int kCvtChunks = 16;  // blocks per array (grid y)

__device__ __forceinline__ void convert_one(const CvtItem& c) {
  const int64_t stride = (int64_t)kCvtChunks * kCvtThreads;
  const int64_t first = (int64_t)blockIdx.y * kCvtThreads + threadIdx.x;
  if (c.to_f64) {
    const float* s = static_cast<const float*>(c.src);
    double* d = static_cast<double*>(c.dst);
    for (int64_t i = first; i < c.count; i += stride) d[i] = (double)s[i];
  } else {
    const double* s = static_cast<const double*>(c.src);
    float* d = static_cast<float*>(c.dst);
    for (int64_t i = first; i < c.count; i += stride) d[i] = (float)s[i];
  }
}

}  // namespace

// Block (x, y): array x, elements y, y + 16 * 256, ...
__global__ __launch_bounds__(kCvtThreads) void k_convert(const CvtItem* items) {
  convert_one(items[blockIdx.x]);
}

__global__ __launch_bounds__(kCvtThreads) void k_convert_list(CvtList list) {
  convert_one(list.it[blockIdx.x]);
}

hipError_t launch_convert(const CvtItem* items, int nitems, hipStream_t stream) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3(nitems, kCvtChunks), dim3(kCvtThreads), 0, stream, items);
  return hipGetLastError();
}

hipError_t launch_convert_list(const CvtList& list, hipStream_t stream) {
  if (list.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_list, dim3(list.n, kCvtChunks), dim3(kCvtThreads), 0, stream, list);
  return hipGetLastError();
}

}  // namespace lqr
