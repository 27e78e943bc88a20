// Persistent batched kernel, register width 48 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(48, 0)
LQR_PERSISTENT_INST(48, 1)
LQR_PERSISTENT_INST(48, 2)
}  // namespace lqr
