// Persistent batched kernel, register width 16 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(16, false)
LQR_PERSISTENT_INST(16, true)
}  // namespace lqr
