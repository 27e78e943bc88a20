// Persistent batched kernel, register width 16 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(16, 0)
LQR_PERSISTENT_INST(16, 1)
LQR_PERSISTENT_INST(16, 2)
}  // namespace lqr
