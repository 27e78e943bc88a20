// Persistent batched kernel, register width 64 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(64, false)
LQR_PERSISTENT_INST(64, true)
}  // namespace lqr
