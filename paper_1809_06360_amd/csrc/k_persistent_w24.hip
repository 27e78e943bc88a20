// Persistent batched kernel, register width 24 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(24, 0)
LQR_PERSISTENT_INST(24, 1)
LQR_PERSISTENT_INST(24, 2)
}  // namespace lqr
