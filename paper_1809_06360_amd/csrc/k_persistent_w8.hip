// Persistent batched kernel, register width 8 (see k_persistent.h): the
// vector-ALU engine only; the width-8 matrix-core variants are not built.
#include "k_persistent.h"

namespace lqr {
LQR_PERSISTENT_INST(8, 0)
}  // namespace lqr
