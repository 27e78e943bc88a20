// Segment-count autotuner and task ordering of batched launches (host code).
#include "lqr_tuner.h"

#include <algorithm>
#include <cmath>
#include <queue>

#include "lqr_cost_model.h"

namespace lqr {

namespace {

double dot4(const double* w, double a, double b, double c, double d) {
  return w[0] * a + w[1] * b + w[2] * c + w[3] * d;
}

// Floating-point operations of one stage (the counts of the kernels' products
// and factorizations): plain Riccati stage, and the extra work of the
// parametric (dual-form) stage.
double flops_plain(double n, double m) {
  return 4 * n * n * n + 6 * n * n * m + 4 * n * m * m + m * m * m / 3.0;
}
double flops_dual_extra(double n, double m) { return 2 * n * n * n + 6 * n * n * m + 2 * n * m * m; }

int max_segments(const TuneInst& in, int slots) {
  if (in.J_fixed > 0) return in.J_fixed;
  if (!in.can_split) return 1;
  return std::max(1, std::min(in.T, 2 * slots));
}

}  // namespace

StageCost stage_cost(int n, int m, int mw, bool mf) {
  const int e = mf ? 1 : 0;
  const double fp = flops_plain(n, m), fd = fp + flops_dual_extra(n, m);
  StageCost c;
  // segments whose resident layout exceeds the LDS run the streamed sweep
  const bool gs = sweep_lds(n, m, true, mw) > kLdsSweepMax;
  c.dual = dot4(gs ? cost::kDualStreamed[e] : cost::kDual[e], 1.0, mw, n, fd / 1e5);
  c.plain = dot4(cost::kPlain[e], 1.0, mw, n, fp / 1e5);
  c.roll = dot4(cost::kRoll[e], 1.0, n, m, (double)n * (n + m) / 1e3);
  c.link = dot4(cost::kLink[e], 1.0, n, (double)n * n / 1e2, (double)n * n * n / 1e4);
  c.task = cost::kTask;
  return c;
}

// Durations of the tasks of one instance: phase-1 segment j, the linking
// solve, phase-3 segment j.
static double dur1(const TuneInst& in, int J, int j, const StageCost& c) {
  const int len = seg_begin(in.T, J, j + 1) - seg_begin(in.T, J, j);
  return c.task + len * (j < J - 1 ? c.dual : c.plain);
}
static double dur2(int J, const StageCost& c) { return c.task + (J - 1) * c.link; }
static double dur3(const TuneInst& in, int J, int j, const StageCost& c) {
  const int len = seg_begin(in.T, J, j + 1) - seg_begin(in.T, J, j);
  return c.task + len * (j < J - 1 ? c.plain + c.roll : c.roll);
}

void instance_cost(const TuneInst& in, int J, const StageCost& c, double* path, double* work) {
  // segments 0 and J-1 are the longest dual and the (shortest) plain one
  const double a1 = J > 1 ? std::max(dur1(in, J, 0, c), dur1(in, J, J - 1, c)) : dur1(in, 1, 0, c);
  const double a3 = J > 1 ? std::max(dur3(in, J, 0, c), dur3(in, J, J - 1, c)) : dur3(in, 1, 0, c);
  *path = a1 + dur2(J, c) + a3;
  const int last = in.T / J;  // length of segment J-1
  const int rest = in.T - last;
  *work = 2 * J * c.task + rest * (c.dual + c.plain + c.roll) + last * (c.plain + c.roll) +
          dur2(J, c);
}

std::vector<TaskItem> order_tasks(const std::vector<TuneInst>& insts, const std::vector<int>& J,
                                  int mw, bool mf, int slots, double* makespan) {
  const int N = (int)insts.size();
  struct Task {
    int inst, seg, phase;
    double dur, blevel, ready;
  };
  std::vector<Task> tasks;
  std::vector<int> first(N + 1, 0);  // tasks of instance i: [first[i], first[i+1])
  for (int i = 0; i < N; ++i) {
    const StageCost c = stage_cost(insts[i].n, insts[i].m, mw, mf);
    const int Ji = J[i];
    first[i] = (int)tasks.size();
    double max3 = 0.0;
    for (int j = 0; j < Ji; ++j) max3 = std::max(max3, dur3(insts[i], Ji, j, c));
    const double d2 = dur2(Ji, c);
    for (int j = 0; j < Ji; ++j) {
      const double d = dur1(insts[i], Ji, j, c);
      tasks.push_back({i, j, 1, d, d + d2 + max3, 0.0});
    }
    tasks.push_back({i, 0, 2, d2, d2 + max3, 0.0});
    for (int j = 0; j < Ji; ++j) {
      const double d = dur3(insts[i], Ji, j, c);
      tasks.push_back({i, j, 3, d, d, 0.0});
    }
  }
  first[N] = (int)tasks.size();
  const int ntasks = (int)tasks.size();

  // ready: highest b-level first; pending: earliest ready time first
  auto by_level = [&](int a, int b) {
    if (tasks[a].blevel != tasks[b].blevel) return tasks[a].blevel < tasks[b].blevel;
    return a > b;
  };
  auto by_ready = [&](int a, int b) {
    if (tasks[a].ready != tasks[b].ready) return tasks[a].ready > tasks[b].ready;
    return by_level(a, b);
  };
  std::priority_queue<int, std::vector<int>, decltype(by_level)> ready(by_level);
  std::priority_queue<int, std::vector<int>, decltype(by_ready)> pending(by_ready);
  std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
  for (int s = 0; s < std::max(1, std::min(slots, ntasks)); ++s) free_at.push(0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < J[i]; ++j) ready.push(first[i] + j);
  std::vector<int> done1(N, 0);
  std::vector<double> fin1(N, 0.0);
  std::vector<TaskItem> order;
  order.reserve(ntasks);
  double end = 0.0;
  while ((int)order.size() < ntasks) {
    const double now = free_at.top();
    free_at.pop();
    while (!pending.empty() && tasks[pending.top()].ready <= now) {
      ready.push(pending.top());
      pending.pop();
    }
    int t;
    if (!ready.empty()) {
      t = ready.top();
      ready.pop();
    } else {
      t = pending.top();
      pending.pop();
    }
    Task& k = tasks[t];
    const double fin = std::max(now, k.ready) + k.dur;
    free_at.push(fin);
    end = std::max(end, fin);
    order.push_back(TaskItem{k.inst, k.seg, k.phase});
    const int i = k.inst;
    if (k.phase == 1) {
      fin1[i] = std::max(fin1[i], fin);
      if (++done1[i] == J[i]) {
        const int t2 = first[i] + J[i];
        tasks[t2].ready = fin1[i];
        pending.push(t2);
      }
    } else if (k.phase == 2) {
      for (int j = 0; j < J[i]; ++j) {
        const int t3 = first[i] + J[i] + 1 + j;
        tasks[t3].ready = fin;
        pending.push(t3);
      }
    }
  }
  if (makespan) *makespan = end;
  return order;
}

std::vector<int> tune_segments(const std::vector<TuneInst>& insts, int mw, bool mf, int slots) {
  const int N = (int)insts.size();
  slots = std::max(1, slots);
  // Per instance: the segment counts at which the predicted critical path
  // reaches a new minimum (scanning J upwards), with their paths and work.
  struct Rec {
    int J;
    double path, work;
  };
  std::vector<std::vector<Rec>> recs(N);
  double lo = 0.0, sum1 = 0.0, hi = 0.0;
  for (int i = 0; i < N; ++i) {
    const StageCost c = stage_cost(insts[i].n, insts[i].m, mw, mf);
    const int jmax = max_segments(insts[i], slots);
    const int jmin = insts[i].J_fixed > 0 ? insts[i].J_fixed : 1;
    for (int J = jmin; J <= jmax; ++J) {
      double p, w;
      instance_cost(insts[i], J, c, &p, &w);
      if (recs[i].empty() || p < recs[i].back().path) recs[i].push_back({J, p, w});
    }
    lo = std::max(lo, recs[i].back().path);
    sum1 += recs[i].front().work;
    hi = std::max(hi, recs[i].front().path);
  }
  hi = std::max(hi, sum1 / slots);
  // smallest segment counts whose predicted paths fit within a makespan M
  auto pick = [&](double M, std::vector<int>* J, double* work) {
    *work = 0.0;
    for (int i = 0; i < N; ++i) {
      const std::vector<Rec>& r = recs[i];
      // paths in r decrease; first record with path <= M
      int a = 0, b = (int)r.size() - 1;
      if (r[b].path > M) a = b;
      while (a < b) {
        const int mid = (a + b) / 2;
        if (r[mid].path <= M) b = mid; else a = mid + 1;
      }
      (*J)[i] = r[a].J;
      *work += r[a].work;
    }
  };
  std::vector<int> J(N, 1);
  double w = 0.0;
  if (hi > lo) {
    for (int it = 0; it < 60 && hi - lo > 1e-3 * lo; ++it) {
      const double mid = 0.5 * (lo + hi);
      pick(mid, &J, &w);
      if (w <= slots * mid) hi = mid; else lo = mid;
    }
  }
  const double bound = hi;
  // Check a few looser targets with the list-scheduling simulation: a
  // looser path target trades critical path for less total work.
  std::vector<int> best;
  double best_t = 0.0;
  for (double f : {1.0, 1.1, 1.25, 1.5, 2.0}) {
    std::vector<int> Jc(N);
    pick(bound * f, &Jc, &w);
    if (!best.empty() && Jc == best) continue;
    double t = 0.0;
    order_tasks(insts, Jc, mw, mf, slots, &t);
    if (best.empty() || t < best_t) {
      best = Jc;
      best_t = t;
    }
  }
  return best;
}

}  // namespace lqr
