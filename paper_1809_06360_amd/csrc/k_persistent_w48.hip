// Persistent batched kernel, register width 48 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(48, false)
LQR_PERSISTENT_INST(48, true)
}  // namespace lqr
