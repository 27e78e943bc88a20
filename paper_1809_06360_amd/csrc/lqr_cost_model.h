// Per-stage cost model of the solver kernels on MI355X (microseconds),
// measured by `python -m paper_1809_06360_amd.calibrate` (single-launch
// phase timings with HIP events, T = 64 stages, non-negative least squares).
//
// Each cost is a non-negative combination of features (see lqr_tuner.cpp):
//   sweeps (dual, dual streamed, plain)  [1, mw, n, flops / 1e5]
//   rollout               [1, n, m, n (n + m) / 1e3]
//   link                  [1, n, n^2 / 1e2, n^3 / 1e4]
// indexed [mf][feature], mf = 1 for the matrix-core product variants.
#pragma once

namespace lqr {
namespace cost {

constexpr double kDual[2][4] = {{9.94823, 0.753842, 0.434153, 0}, {0, 0.406604, 0.3238, 1.45567}};
constexpr double kDualStreamed[2][4] = {{0, 0, 0, 0}, {15.0186, 0.76935, 0.121546, 0.896429}};
constexpr double kPlain[2][4] = {{7.13742, 0.669526, 0.32809, 0}, {0.200634, 0.587989, 0.106433, 1.43635}};
constexpr double kRoll[2][4] = {{3.13653, 0.00860262, 0, 0}, {2.90969, 0, 0, 0.303048}};
constexpr double kLink[2][4] = {{5.17158, 0.883042, 0, 0}, {0, 0.39376, 1.30191, 0}};
constexpr double kTask = 3.0;

}  // namespace cost
}  // namespace lqr
