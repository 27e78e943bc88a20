// Engine dispatch of the large-state sweep kernels (instantiated in
// k_big_e1.hip and k_big_e2.hip).
#include "k_big.h"

namespace lqr {

hipError_t launch_big_sweep(const InstDesc& d, int kind, int eng, size_t lds, hipStream_t stream) {
  if (eng == 1) return launch_big_sweep_e<1>(d, kind, lds, stream);
  if (eng == 2) return launch_big_sweep_e<2>(d, kind, lds, stream);
  return hipErrorInvalidValue;
}

}  // namespace lqr
