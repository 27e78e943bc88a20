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

constexpr double kDual[2][4] = {{5.29604, 1.07675, 0.455264, 0}, {0, 0.642568, 0.1632, 1.87494}};
constexpr double kDualStreamed[2][4] = {{0, 0, 0, 0}, {21.2248, 0.855609, 0, 1.06303}};
constexpr double kPlain[2][4] = {{2.85994, 0.947504, 0.321034, 0.190963}, {0, 0.651159, 0, 2.36462}};
constexpr double kRoll[2][4] = {{0.671614, 0.129015, 0.0993282, 0.201129}, {1.98254, 0.0762027, 0.0843853, 0.571415}};
constexpr double kLink[2][4] = {{3.72888, 1.85297, 0, 6.82112}, {46.5308, 0, 0, 10.046}};
constexpr double kTask = 3.0;

}  // namespace cost
}  // namespace lqr
