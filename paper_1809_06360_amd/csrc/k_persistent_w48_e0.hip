// Persistent batched kernel, register width 48, vector-ALU engine (see
// k_persistent.h; one translation unit per variant so the library builds in
// parallel).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(48, 0)
}  // namespace lqr
