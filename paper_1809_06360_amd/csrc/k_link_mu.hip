// Link multipliers of a solved instance: mu_j = P x + p at each link point
// t_{j+1} (Sec. II-A link equation; Sec. II-B, eq. mu), one workgroup per link
// point, from the solve's outputs.
#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_link_mu(int n, int Tn, int J, const T* P, const T* p,
                                                      const T* x, T* mu) {
  extern __shared__ double smem[];
  T* sx = reinterpret_cast<T*>(smem);
  const int j = blockIdx.x;
  const int t = seg_begin(Tn, J, j + 1);
  const T* Pt = P + (size_t)t * n * n;
  const T* pt = p + (size_t)t * n;
  const T* xt = x + (size_t)t * n;
  for (int i = threadIdx.x; i < n; i += kThreads) sx[i] = xt[i];
  __syncthreads();
  T* out = mu + (size_t)j * n;
  gemv2(n, n, Pt, n, sx, 0, sx, 0, sx, [=](int i, T v) { out[i] = pt[i] + v; });
}

hipError_t launch_link_mu(int n, int T, int J, const void* P, const void* p, const void* x, void* mu,
                          bool f32, hipStream_t stream) {
  if (J < 2) return hipSuccess;
  const size_t lds = 128 * sizeof(double);
  if (f32)
    hipLaunchKernelGGL(k_link_mu<float>, dim3(J - 1), dim3(kThreads), lds, stream, n, T, J,
                       static_cast<const float*>(P), static_cast<const float*>(p),
                       static_cast<const float*>(x), static_cast<float*>(mu));
  else
    hipLaunchKernelGGL(k_link_mu<double>, dim3(J - 1), dim3(kThreads), lds, stream, n, T, J,
                       static_cast<const double*>(P), static_cast<const double*>(p),
                       static_cast<const double*>(x), static_cast<double*>(mu));
  return hipGetLastError();
}

}  // namespace lqr
