// The phase-1 sweep kernels of the FP64 matrix-core engine, all register widths
// (one translation unit per kernel and engine; see k_sweeps.h).
#include "k_sweeps.h"

namespace lqr {
LQR_SWEEP_INST(kSweepPhase1, 1)
}  // namespace lqr
