// The plain serial sweep kernels of the FP32 matrix-core engine, all register widths
// (one translation unit per kernel and engine; see k_sweeps.h).
#include "k_sweeps.h"

namespace lqr {
LQR_SWEEP_INST(kSweepSerial, 2)
}  // namespace lqr
