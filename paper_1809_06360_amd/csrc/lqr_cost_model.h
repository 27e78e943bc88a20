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

constexpr double kDual[2][4] = {{9.7286, 0.730256, 0.429983, 0}, {0, 0.356084, 0.357421, 1.40153}};
constexpr double kDualStreamed[2][4] = {{0, 0, 0, 0}, {18.2212, 0.670574, 0.102654, 0.879499}};
constexpr double kPlain[2][4] = {{7.14759, 0.647563, 0.327282, 0}, {0, 0.56655, 0.11784, 1.3803}};
constexpr double kRoll[2][4] = {{3.00464, 0.00973967, 0, 0}, {2.82051, 0, 0.00239331, 0.297841}};
constexpr double kLink[2][4] = {{4.32689, 1.86254, 0, 6.81954}, {46.8948, 0, 0, 10.0985}};
constexpr double kTask = 3.0;

}  // namespace cost
}  // namespace lqr
