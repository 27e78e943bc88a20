// Persistent batched kernel, register width 8 (see k_persistent.h).
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(8, 0)
LQR_PERSISTENT_INST(8, 1)
LQR_PERSISTENT_INST(8, 2)
}  // namespace lqr
