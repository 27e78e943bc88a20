// Per-stage cost model of the solver kernels on MI355X (microseconds),
// measured by `python -m paper_1809_06360_amd.calibrate` (single-launch
// phase timings with HIP events, T = 64 stages, non-negative least squares).
//
// Each cost is a non-negative combination of features (see lqr_tuner.cpp):
//   sweeps (dual, plain)  [1, mw, n, flops / 1e5]
//   rollout               [1, n, m, n (n + m) / 1e3]
//   link                  [1, n, n^2 / 1e2, n^3 / 1e4]
// indexed [mf][feature], mf = 1 for the matrix-core product variants.
#pragma once

namespace lqr {
namespace cost {

constexpr double kDual[2][4] = {{5.02026, 1.0647, 0.470868, 0}, {0, 0.610893, 0.311542, 1.37193}};
constexpr double kPlain[2][4] = {{3.0596, 0.94327, 0.319475, 0.280658}, {0.299484, 0.685929, 0.0832989, 2.03126}};
constexpr double kRoll[2][4] = {{0.672119, 0.12952, 0.0999225, 0.208706}, {2.49015, 0.0525247, 0.079339, 0.812195}};
constexpr double kLink[2][4] = {{3.7351, 1.85928, 0, 6.90074}, {50.0656, 0, 0, 9.24858}};
constexpr double kTask = 3.0;

}  // namespace cost
}  // namespace lqr
