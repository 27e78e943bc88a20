// Segment-count autotuner and task ordering of batched launches (host code).
//
// The cost of every task is predicted by a per-stage model of the kernels
// (lqr_cost_model.h, fitted to timings measured on the device). The tuner
// picks each instance's segment count J_i to minimise the predicted makespan
// of the whole batch on the device's resident workgroup slots, and orders the
// tasks of the persistent launch by a list-scheduling simulation.
#pragma once

#include <vector>

#include "lqr_layout.h"

namespace lqr {

struct TuneInst {
  int n, m, T;
  int J_fixed;     // > 0: caller's segment count, kept
  bool can_split;  // the dual sweep and the linking solve fit this instance
};

// Predicted per-stage (sweep, rollout) and per-boundary (link) costs in
// microseconds for an instance run by the kernel variant of register width
// mw with product engine mf.
struct StageCost {
  double dual, plain, roll, link, task;
};
StageCost stage_cost(int n, int m, int mw, bool mf);

// Predicted critical path and total work (microseconds) of one instance
// split into J segments.
void instance_cost(const TuneInst& in, int J, const StageCost& c, double* path, double* work);

// Segment counts for a batch sharing one kernel variant (mw, mf) on `slots`
// resident workgroups.
std::vector<int> tune_segments(const std::vector<TuneInst>& insts, int mw, bool mf, int slots);

// Task order of the persistent launch (a topological order of the task
// dependencies) for the given segment counts; *makespan receives the
// simulated makespan in microseconds.
std::vector<TaskItem> order_tasks(const std::vector<TuneInst>& insts, const std::vector<int>& J,
                                  int mw, bool mf, int slots, double* makespan);

}  // namespace lqr
