// Persistent batched kernel, register width 64 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(64, 0)
LQR_PERSISTENT_INST(64, 1)
LQR_PERSISTENT_INST(64, 2)
}  // namespace lqr
