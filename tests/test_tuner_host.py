"""Host-side checks of the batched planner's task ordering (no GPU).

The persistent batched kernel is free of deadlock only if its task table is a
topological order of the dependencies (every phase-1 task of an instance
before its phase-2 task, which comes before its phase-3 tasks) and holds each
task exactly once. A small C++ driver compiled with g++ against the planner's
own source checks this on random batches, and that the simulated makespan is
no smaller than the two lower bounds (total work / slots, longest path).
"""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_06360_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <random>
#include <vector>
#include "lqr_tuner.h"
using namespace lqr;
int main() {
  std::mt19937 rng(7);
  int bad = 0;
  for (int trial = 0; trial < 60; ++trial) {
    const int N = 1 + rng() % 300;
    std::vector<TuneInst> in(N);
    int maxm = 1;
    bool mf = false;
    for (auto& x : in) {
      x.n = 1 + rng() % 64; x.m = 1 + rng() % 32; x.T = 1 + rng() % 600;
      x.J_fixed = (rng() % 4 == 0) ? 1 + rng() % x.T : 0;
      x.can_split = rng() % 5 != 0;
      if (!x.can_split && x.J_fixed > 1) x.J_fixed = 1;
      maxm = std::max(maxm, x.m);
      mf = mf || x.n >= 32;
    }
    const int mw = pad_rows(maxm);
    const int slots = 256 * (1 + rng() % 2);
    std::vector<int> J = tune_segments(in, mw, mf, slots);
    double mk = 0.0, work = 0.0, path = 0.0;
    std::vector<TaskItem> ord = order_tasks(in, J, mw, mf, slots, &mk);
    size_t expect = 0;
    for (int i = 0; i < N; ++i) {
      if (J[i] < 1 || J[i] > in[i].T) { std::printf("J out of range\n"); ++bad; }
      if (in[i].J_fixed > 0 && J[i] != in[i].J_fixed) { std::printf("fixed J changed\n"); ++bad; }
      if (!in[i].can_split && J[i] != 1) { std::printf("split an unsplittable instance\n"); ++bad; }
      expect += 2 * J[i] + 1;
      double p, w;
      instance_cost(in[i], J[i], stage_cost(in[i].n, in[i].m, mw, mf), &p, &w);
      work += w; path = std::max(path, p);
    }
    if (ord.size() != expect) { std::printf("task count %zu != %zu\n", ord.size(), expect); ++bad; }
    std::vector<int> d1(N, 0), d2(N, 0);
    std::vector<std::vector<int>> seen1(N), seen3(N);
    for (int i = 0; i < N; ++i) { seen1[i].assign(J[i], 0); seen3[i].assign(J[i], 0); }
    for (const TaskItem& t : ord) {
      const int i = t.inst;
      if (i < 0 || i >= N || t.seg < 0 || t.seg >= J[i]) { std::printf("bad task\n"); ++bad; continue; }
      if (t.phase == 1) { if (seen1[i][t.seg]++) { std::printf("dup p1\n"); ++bad; } ++d1[i]; }
      else if (t.phase == 2) { if (d1[i] != J[i] || d2[i]++) { std::printf("p2 early/dup\n"); ++bad; } }
      else if (t.phase == 3) { if (d2[i] != 1 || seen3[i][t.seg]++) { std::printf("p3 early/dup\n"); ++bad; } }
      else { std::printf("bad phase\n"); ++bad; }
    }
    if (mk + 1e-6 < work / slots || mk + 1e-6 < path) { std::printf("makespan below bound\n"); ++bad; }
  }
  std::printf("bad=%d\n", bad);
  return bad != 0;
}
"""


def test_task_order_is_topological_and_complete(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, "-o", str(exe), str(src),
                           os.path.join(CSRC, "lqr_tuner.cpp")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:]
    assert "bad=0" in out.stdout
