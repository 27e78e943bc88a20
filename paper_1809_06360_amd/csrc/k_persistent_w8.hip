// Persistent batched kernel, register width 8 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(8, false)
LQR_PERSISTENT_INST(8, true)
}  // namespace lqr
