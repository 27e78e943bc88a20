// Large-state sweep kernels of the FP64 matrix-core engine (see k_big.h).
#include "k_big.h"

namespace lqr {
template hipError_t launch_big_sweep_e<1>(const InstDesc&, int, size_t, hipStream_t);
}  // namespace lqr
