// Persistent batched kernel, register width 32 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(32, 0)
LQR_PERSISTENT_INST(32, 1)
LQR_PERSISTENT_INST(32, 2)
}  // namespace lqr
