// C-ABI entry points: argument validation, the segment planner, workspace
// carve-out and kernel launches. No device memory is allocated here; every
// launch goes to the caller's stream and nothing synchronises it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "lqr_kernels.h"
#include "lqr_launch.h"
#include "lqr_layout.h"
#include "lqr_tuner.h"
#include "mi355lqr.h"

namespace lqr {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// LDS a gfx950 workgroup may allocate. Plans (segment counts, workspace
// sizes) are computed against this architectural constant so they do not
// depend on the machine; launches also check the device's reported limit.
constexpr size_t kLdsGfx950 = 160 * 1024;

// Largest dynamic LDS allocation a workgroup may ask for on the current device.
size_t device_lds_bytes() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  size_t bytes = 64 * 1024;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    bytes = (size_t)v;
  cache[dev] = bytes;
  return bytes;
}

// Compute units of an MI355X; the planner sizes batches against it.
constexpr int kComputeUnits = 256;

// Whether an instance can be split into segments: the dual sweep and the
// linking solve must fit the kernels' register and LDS budgets.
bool can_split(int n, int m, int mw, int nw) {
  return n <= 64 && 2 * n + 1 <= 256 && sweep_fits_regs(n, m, true) &&
         dual_lds(n, m, mw) <= kLdsGfx950 && couple_lds(n, nw) <= kLdsGfx950;
}

struct InstPlan {
  int J;
  size_t ws_off;   // bytes from the workspace base
  size_t ws_bytes;
  size_t stage_off = 0;  // FP32 mode: FP64 staging of the instance's inputs and outputs
};

// Workspace regions of a problem set. They depend only on the instances'
// n, m, T (not on the options), so lqr_solve_batched and lqr_backward on the
// same problem set agree on them:
//   [0, adj_cap)                   lqr_backward's uploaded plan
//   [fwd_off, fwd_off + fwd_cap)   lqr_solve_batched's uploaded plan
//   [scratch_off, ...)             per-call scratch (either call's)
// Each plan region is sized for its largest possible table: every instance
// split into T segments, and the FP32 conversion lists.
struct Regions {
  size_t adj_cap = 0, fwd_off = 0, fwd_cap = 0, scratch_off = 0;
};

// FP32 staging conversions per instance in a batched plan's table: up to 9
// inputs in, 8 outputs out; in the adjoint's table: 10 in, 9 out.
constexpr int kCvtPerInst = 17;
constexpr int kAdjCvtPerInst = 19;

int adj_blocks(int T) { return (T + 1 + kAdjStages - 1) / kAdjStages; }

Regions regions_of(const lqr_problem_t* probs, int batch) {
  size_t sum_t = 0, nb = 0;
  for (int i = 0; i < batch; ++i) {
    sum_t += (size_t)std::max(probs[i].T, 1);
    nb += (size_t)adj_blocks(std::max(probs[i].T, 1));
  }
  Regions r;
  r.adj_cap = align_up(sizeof(AdjDesc) * (size_t)batch) + align_up(sizeof(int2) * nb) +
              align_up(sizeof(CvtItem) * (size_t)kAdjCvtPerInst * batch);
  r.fwd_off = r.adj_cap;
  r.fwd_cap = align_up(sizeof(InstDesc) * (size_t)batch) + align_up(sizeof(WorkItem) * sum_t) +
              align_up(sizeof(TaskItem) * (2 * sum_t + (size_t)batch)) +
              align_up(sizeof(CvtItem) * (size_t)kCvtPerInst * batch);
  r.scratch_off = r.fwd_off + r.fwd_cap;
  return r;
}

// Workspace layout of a forward call: in the batched-plan region, descriptor
// table | phase-1/3 work items (phased launches) | persistent task table |
// FP32 conversion list (together the uploaded plan, table_bytes from
// table_off); in the scratch region, synchronisation words | FP32 staging |
// per-instance scratch. Offsets are from the workspace base.
struct BatchPlan {
  std::vector<InstPlan> inst;
  std::vector<TaskItem> tasks;  // persistent launch order (parallel algorithm)
  double est_us = 0.0;          // predicted makespan of the persistent launch
  Regions reg;
  size_t table_off = 0, items_off = 0, tasks_off = 0, cvt_off = 0, sync_off = 0;
  size_t table_bytes = 0;       // bytes of the uploaded plan
  size_t total_bytes = 0;
  int nitems = 0;
  int max_n = 1, max_m = 1;
  bool big = false;  // one instance with 65..128 states: the large-state kernels
  size_t lds1 = 0, lds2 = 0, lds3 = 0, lds_serial = 0, lds_persist = 0;
};

bool is_serial(const lqr_options_t* o) { return o && o->algo == LQR_ALGO_SERIAL; }
bool is_phased(const lqr_options_t* o) { return o && (o->flags & LQR_FLAG_PHASED); }
bool is_smoothed(const lqr_options_t* o) { return o && (o->flags & LQR_FLAG_SMOOTHED); }
bool is_mixed(const lqr_options_t* o) { return o && o->precision == LQR_PREC_MIXED; }
bool is_f32(const lqr_options_t* o) { return o && o->precision == LQR_PREC_FP32; }
// Product engine of the large-state kernels: FP32 matrix cores in the mixed and
// FP32 modes, FP64 matrix cores otherwise.
int big_engine(const lqr_options_t* o) { return (is_mixed(o) || is_f32(o)) ? 2 : 1; }

// Every instance within the small-size recursion (n, m <= 16; k_small.hip).
bool small_enough(const BatchPlan& p) { return !p.big && p.max_n <= kSmallMax && p.max_m <= kSmallMax; }

lqr_status_t check_options(const lqr_options_t* o) {
  if (!o) return LQR_SUCCESS;
  if (o->flags & ~(uint32_t)(LQR_FLAG_PHASED | LQR_FLAG_SMOOTHED)) return LQR_ERR_INVALID_ARG;
  if ((o->flags & LQR_FLAG_SMOOTHED) && o->algo == LQR_ALGO_SERIAL) return LQR_ERR_INVALID_ARG;
  if (o->algo != LQR_ALGO_PARALLEL && o->algo != LQR_ALGO_SERIAL) return LQR_ERR_INVALID_ARG;
  if (o->precision != LQR_PREC_FP64 && o->precision != LQR_PREC_MIXED &&
      o->precision != LQR_PREC_FP32)
    return LQR_ERR_INVALID_ARG;
  return LQR_SUCCESS;
}

lqr_status_t check_dims(const lqr_problem_t& p) {
  if (p.n < 1 || p.m < 1 || p.T < 1) return LQR_ERR_INVALID_ARG;
  if (p.segments < 0 || p.segments > p.T) return LQR_ERR_INVALID_ARG;
  return LQR_SUCCESS;
}

lqr_status_t check_pointers(const lqr_problem_t& p) {
  if (!p.A || !p.B || !p.c || !p.Q || !p.q || !p.R || !p.r || !p.x0) return LQR_ERR_INVALID_ARG;
  if (!p.K || !p.k || !p.x || !p.u || !p.info) return LQR_ERR_INVALID_ARG;
  if (p.lam && (!p.P || !p.p)) return LQR_ERR_INVALID_ARG;
  return LQR_SUCCESS;
}

// Resident workgroups the tuner plans for: one per compute unit. The
// persistent kernel holds every task type, which takes more than 256 VGPRs
// per lane, so one 256-thread workgroup fills a compute unit whatever its LDS.
int planned_slots(size_t /*lds*/) { return kComputeUnits; }

// Segments of a large-state instance when the caller leaves the choice to the
// planner: about 16 stages each (the dual sweep's extra work against the
// logarithmic-depth linking solve), at most 256.
int big_segments(int T) { return std::max(1, std::min(256, std::min(T, (T + 8) / 16))); }

// Plan of one instance with 65..128 states (at most 64 inputs): the
// large-state kernels, one 256-thread workgroup per segment.
lqr_status_t build_big_plan(const lqr_problem_t& p, const lqr_options_t* opts, BatchPlan* plan) {
  plan->big = true;
  plan->max_n = p.n;
  plan->max_m = p.m;
  const int J = is_serial(opts) ? 1 : (p.segments > 0 ? p.segments : big_segments(p.T));
  plan->inst[0].J = J;
  plan->nitems = J;
  plan->lds1 = plan->lds3 = plan->lds_serial = big_sweep_lds();
  plan->lds2 = big_link_lds();
  plan->reg = regions_of(&p, 1);
  plan->table_off = plan->reg.fwd_off;
  plan->items_off = plan->tasks_off = plan->cvt_off = plan->table_off;
  plan->table_bytes = 0;
  plan->sync_off = plan->reg.scratch_off;
  size_t off = plan->sync_off + align_up(sizeof(int32_t) * sync_words(1));
  if (is_f32(opts)) {
    plan->inst[0].stage_off = off;
    off += align_up((stage_in_doubles(p.n, p.m, p.T) + stage_out_doubles(p.n, p.m, p.T)) * sizeof(double));
  }
  const size_t bytes = align_up(big_ws_doubles(p.n, p.m, J) * sizeof(double)) +
                       align_up(sizeof(int32_t) * fail_words(J));
  plan->inst[0].ws_off = off;
  plan->inst[0].ws_bytes = bytes;
  plan->total_bytes = off + bytes;
  return LQR_SUCCESS;
}

lqr_status_t build_plan(const lqr_problem_t* probs, int batch, const lqr_options_t* opts,
                        BatchPlan* plan) {
  lqr_status_t st = check_options(opts);
  if (st != LQR_SUCCESS) return st;
  const size_t lds_max = kLdsGfx950;
  const bool serial = is_serial(opts);
  plan->inst.resize(batch);
  // The batch's largest dimensions pick the kernel variants, whose register
  // widths fix the LDS layouts; segment counts are planned against them.
  for (int i = 0; i < batch; ++i) {
    const lqr_problem_t& p = probs[i];
    if ((st = check_dims(p)) != LQR_SUCCESS) return st;
    if (p.n > 64 || p.m > 64) {
      // the large-state kernels: single instances of up to 128 states and 64 inputs
      if (!is_big(p.n, p.m) || batch != 1) return LQR_ERR_UNSUPPORTED;
      return build_big_plan(p, opts, plan);
    }
    plan->max_n = std::max(plan->max_n, p.n);
    plan->max_m = std::max(plan->max_m, p.m);
  }
  const int eng = launch_engine(plan->max_n, is_mixed(opts) || is_f32(opts));
  const int mw = pad_rows(kernel_width(plan->max_m, eng));
  const bool mf = eng != 0;
  // linking-solve width: that of the phased kernel or of the persistent one
  const int nw = std::max(pad_rows(plan->max_n), persist_nw(mf));
  std::vector<TuneInst> tin(batch);
  size_t lds_guess = 0;
  for (int i = 0; i < batch; ++i) {
    const lqr_problem_t& p = probs[i];
    const bool split = !serial && can_split(p.n, p.m, mw, nw);
    if (p.segments > 1 && !split && !serial) return LQR_ERR_UNSUPPORTED;
    tin[i] = TuneInst{p.n, p.m, p.T, serial ? 1 : p.segments, split};
    lds_guess = std::max(lds_guess, sweep_lds(p.n, p.m, false, mw));
    if (split) lds_guess = std::max(lds_guess, dual_lds(p.n, p.m, mw));
    if (split) lds_guess = std::max(lds_guess, couple_lds(p.n, nw));
  }
  std::vector<int> J = tune_segments(tin, mw, mf, planned_slots(lds_guess));
  int items = 0;
  for (int i = 0; i < batch; ++i) {
    plan->inst[i].J = J[i];
    items += J[i];
  }
  for (int i = 0; i < batch; ++i) {
    const lqr_problem_t& p = probs[i];
    const int Ji = J[i];
    const size_t plain = sweep_lds(p.n, p.m, false, mw);
    if (plain > lds_max || !sweep_fits_regs(p.n, p.m, false)) return LQR_ERR_UNSUPPORTED;
    plan->lds_serial = std::max(plan->lds_serial, std::max(plain, rollout_lds(p.n, p.m)));
    // phase 1 runs the parametric sweep on segments j < J-1 and the plain
    // recursion on the last one; the streamed sweep can need less than the latter
    plan->lds1 = std::max(plan->lds1, Ji > 1 ? std::max(dual_lds(p.n, p.m, mw), plain) : plain);
    plan->lds2 = std::max(plan->lds2, couple_lds(p.n, pad_rows(plan->max_n)));
    if (batch == 1 && use_link_tree(p.n, Ji))
      plan->lds2 = std::max(plan->lds2, link_tree_lds(p.n, pad_rows(p.n)));
    plan->lds3 = std::max(plan->lds3, std::max(plain, rollout_lds(p.n, p.m)));
    if (!serial) plan->lds_persist = std::max(plan->lds_persist, couple_lds(p.n, persist_nw(mf)));
  }
  if (!serial) {
    plan->lds_persist = std::max(plan->lds_persist, std::max(plan->lds1, plan->lds3));
    if (plan->lds_persist + 32 > lds_max) return LQR_ERR_UNSUPPORTED;
    plan->tasks = order_tasks(tin, J, mw, mf, planned_slots(plan->lds_persist), &plan->est_us);
  }
  plan->nitems = items;
  plan->reg = regions_of(probs, batch);
  plan->table_off = plan->reg.fwd_off;
  plan->items_off = plan->table_off + align_up(sizeof(InstDesc) * (size_t)batch);
  plan->tasks_off = plan->items_off + align_up(sizeof(WorkItem) * (size_t)items);
  plan->cvt_off = plan->tasks_off + align_up(sizeof(TaskItem) * plan->tasks.size());
  plan->table_bytes = plan->cvt_off - plan->table_off +
                      (is_f32(opts) ? align_up(sizeof(CvtItem) * (size_t)kCvtPerInst * batch) : 0);
  if (plan->table_bytes > plan->reg.fwd_cap) return LQR_ERR_INVALID_ARG;  // cannot happen: J <= T
  plan->sync_off = plan->reg.scratch_off;
  size_t off = plan->sync_off + align_up(sizeof(int32_t) * sync_words(batch));
  if (is_f32(opts))
    for (int i = 0; i < batch; ++i) {
      const lqr_problem_t& p = probs[i];
      plan->inst[i].stage_off = off;
      off += align_up((stage_in_doubles(p.n, p.m, p.T) + stage_out_doubles(p.n, p.m, p.T)) *
                      sizeof(double));
    }
  for (int i = 0; i < batch; ++i) {
    const lqr_problem_t& p = probs[i];
    const int Ji = J[i];
    const size_t bytes = align_up(ws_doubles(p.n, Ji) * sizeof(double)) +
                         align_up(sizeof(int32_t) * fail_words(Ji));
    plan->inst[i].ws_off = off;
    plan->inst[i].ws_bytes = bytes;
    off += bytes;
  }
  plan->total_bytes = off;
  return LQR_SUCCESS;
}

// Plans are cached by (options, per-instance n, m, T, segments): the tuner's
// search and the task ordering run once per distinct batch shape.
std::mutex g_cache_mu;
std::map<std::vector<int32_t>, BatchPlan> g_cache;

lqr_status_t make_plan(const lqr_problem_t* probs, int batch, const lqr_options_t* opts,
                       BatchPlan* plan) {
  if (!probs || batch < 1) return LQR_ERR_INVALID_ARG;
  std::vector<int32_t> key;
  key.reserve(4 + 4 * (size_t)batch);
  key.push_back(batch);
  key.push_back(opts ? (int32_t)opts->precision : 0);
  key.push_back(opts ? (int32_t)opts->algo : 0);
  key.push_back(opts ? (int32_t)opts->flags : 0);
  for (int i = 0; i < batch; ++i) {
    key.push_back(probs[i].n);
    key.push_back(probs[i].m);
    key.push_back(probs[i].T);
    key.push_back(probs[i].segments);
  }
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *plan = it->second;
      return LQR_SUCCESS;
    }
  }
  BatchPlan fresh;
  lqr_status_t st = build_plan(probs, batch, opts, &fresh);
  if (st != LQR_SUCCESS) return st;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  if (g_cache.size() >= 64) g_cache.clear();
  g_cache[key] = fresh;
  *plan = fresh;
  return LQR_SUCCESS;
}

lqr_status_t check_device(const BatchPlan& plan) {
  const size_t lim = device_lds_bytes();
  const size_t need = std::max(std::max(plan.lds1, plan.lds2),
                               std::max(std::max(plan.lds3, plan.lds_serial), plan.lds_persist + 32));
  return need <= lim ? LQR_SUCCESS : LQR_ERR_UNSUPPORTED;
}

// Adjoint layout: in the adjoint-plan region, AdjDesc table | stage-block
// table | FP32 conversion list (the uploaded plan, table_bytes from offset 0);
// in the scratch region, per-instance scratch and FP32 staging.
struct AdjPlan {
  size_t table_bytes = 0, blocks_off = 0, cvt_off = 0, total_bytes = 0;
  int nblocks = 0;
  Regions reg;
  std::vector<size_t> ws_off;
  std::vector<size_t> stage_off;  // FP32 mode staging per instance
  size_t lds = 0;
};

// FP32 adjoint staging per instance (doubles): A, B, K, P, chol, x, u, lam,
// dl_dx, dl_du in; dA, dB, dc, dQ, dq, dR, dr, dS, dx0 out.
size_t adj_stage_doubles(int n, int m, int T) {
  const size_t t = T, t1 = (size_t)T + 1;
  const size_t in = t * n * n + t * n * m + t * m * n + t1 * n * n + t * m * m + 2 * t1 * n + t * m +
                    t1 * n + t * m;
  const size_t out = t * n * n + t * n * m + t * n + t1 * n * n + t1 * n + t * m * m + t * m +
                     t * m * n + n;
  return in + out;
}
lqr_status_t make_adj_plan(const lqr_problem_t* probs, int batch, AdjPlan* ap, bool f32) {
  if (!probs || batch < 1) return LQR_ERR_INVALID_ARG;
  ap->ws_off.resize(batch);
  ap->stage_off.assign(batch, 0);
  int nb = 0;
  for (int i = 0; i < batch; ++i) {
    lqr_status_t st = check_dims(probs[i]);
    if (st != LQR_SUCCESS) return st;
    if (probs[i].m > 64) return LQR_ERR_UNSUPPORTED;
    nb += adj_blocks(probs[i].T);
    ap->lds = std::max(ap->lds, adj_lds(probs[i].n, probs[i].m));
    if (probs[i].n <= kSmallMax && probs[i].m <= kSmallMax)
      ap->lds = std::max(ap->lds, adjoint_small_lds());
  }
  ap->nblocks = nb;
  ap->reg = regions_of(probs, batch);
  ap->blocks_off = align_up(sizeof(AdjDesc) * (size_t)batch);
  ap->cvt_off = ap->blocks_off + align_up(sizeof(int2) * (size_t)nb);
  ap->table_bytes = ap->cvt_off + (f32 ? align_up(sizeof(CvtItem) * (size_t)kAdjCvtPerInst * batch) : 0);
  if (ap->table_bytes > ap->reg.adj_cap) return LQR_ERR_INVALID_ARG;  // cannot happen
  size_t off = ap->reg.scratch_off;
  for (int i = 0; i < batch; ++i) {
    ap->ws_off[i] = off;
    off += align_up(adj_ws_doubles(probs[i].n, probs[i].m, probs[i].T) * sizeof(double));
    if (f32) {
      ap->stage_off[i] = off;
      off += align_up(adj_stage_doubles(probs[i].n, probs[i].m, probs[i].T) * sizeof(double));
    }
  }
  ap->total_bytes = off;
  return LQR_SUCCESS;
}

InstDesc make_desc(const lqr_problem_t& p, int J, char* ws_base, size_t ws_off) {
  InstDesc d;
  d.n = p.n;
  d.m = p.m;
  d.T = p.T;
  d.J = J;
  d.A = static_cast<const double*>(p.A);
  d.B = static_cast<const double*>(p.B);
  d.c = static_cast<const double*>(p.c);
  d.Q = static_cast<const double*>(p.Q);
  d.q = static_cast<const double*>(p.q);
  d.R = static_cast<const double*>(p.R);
  d.r = static_cast<const double*>(p.r);
  d.S = static_cast<const double*>(p.S);
  d.x0 = static_cast<const double*>(p.x0);
  d.K = static_cast<double*>(p.K);
  d.k = static_cast<double*>(p.k);
  d.P = static_cast<double*>(p.P);
  d.p = static_cast<double*>(p.p);
  d.x = static_cast<double*>(p.x);
  d.u = static_cast<double*>(p.u);
  d.lam = static_cast<double*>(p.lam);
  d.chol = static_cast<double*>(p.chol);
  d.info = p.info;
  d.ws = reinterpret_cast<double*>(ws_base + ws_off);
  const size_t wsd = is_big(p.n, p.m) ? big_ws_doubles(p.n, p.m, J) : ws_doubles(p.n, J);
  d.fail = reinterpret_cast<int32_t*>(ws_base + ws_off + align_up(wsd * sizeof(double)));
  return d;
}

// FP32 mode: the descriptor of an instance whose arrays are the FP64 staging
// copies at `stage` (inputs A..x0, then outputs K..chol, see stage_in_doubles),
// and the conversions that fill the inputs and return the requested outputs.
InstDesc make_desc_f32(const lqr_problem_t& p, int J, char* ws_base, size_t ws_off, size_t stage,
                       CvtItem* cin, int* nin, CvtItem* cout, int* nout) {
  InstDesc d = make_desc(p, J, ws_base, ws_off);
  const int n = p.n, m = p.m, T = p.T;
  double* q = reinterpret_cast<double*>(ws_base + stage);
  *nin = 0;
  *nout = 0;
  auto in = [&](const void* user, size_t count) -> const double* {
    double* dst = q;
    q += count;
    if (!user) return nullptr;
    cin[(*nin)++] = CvtItem{user, dst, (int64_t)count, 1, 0};
    return dst;
  };
  d.A = in(p.A, (size_t)T * n * n);
  d.B = in(p.B, (size_t)T * n * m);
  d.c = in(p.c, (size_t)T * n);
  d.Q = in(p.Q, (size_t)(T + 1) * n * n);
  d.q = in(p.q, (size_t)(T + 1) * n);
  d.R = in(p.R, (size_t)T * m * m);
  d.r = in(p.r, (size_t)T * m);
  d.S = in(p.S, (size_t)T * m * n);
  d.x0 = in(p.x0, (size_t)n);
  auto out = [&](void* user, size_t count) -> double* {
    double* src = q;
    q += count;
    if (!user) return nullptr;
    cout[(*nout)++] = CvtItem{src, user, (int64_t)count, 0, 0};
    return src;
  };
  d.K = out(p.K, (size_t)T * m * n);
  d.k = out(p.k, (size_t)T * m);
  d.P = out(p.P, (size_t)(T + 1) * n * n);
  d.p = out(p.p, (size_t)(T + 1) * n);
  d.x = out(p.x, (size_t)(T + 1) * n);
  d.u = out(p.u, (size_t)T * m);
  d.lam = out(p.lam, (size_t)(T + 1) * n);
  d.chol = out(p.chol, (size_t)T * m * m);
  return d;
}

// Host copies of the plans uploaded into each workspace (keyed by its
// address), so that a call under stream capture can verify that the plan it
// needs is resident. `layout` is the dims key of the problem set whose regions
// hold them. A host buffer handed to hipMemcpyAsync stays alive until an
// event recorded after the copy has completed (retired buffers are released
// by later calls once their copies are done).
struct Upload {
  std::vector<char> bytes;
  hipEvent_t done = nullptr;
};
struct WsPlans {
  std::vector<int32_t> layout;
  std::unique_ptr<Upload> fwd, adj;
};
std::mutex g_plan_mu;
std::map<void*, WsPlans> g_plans;
std::vector<std::unique_ptr<Upload>> g_retired;

std::vector<int32_t> layout_key(const lqr_problem_t* probs, int batch) {
  std::vector<int32_t> key;
  key.reserve(1 + 3 * (size_t)batch);
  key.push_back(batch);
  for (int i = 0; i < batch; ++i) {
    key.push_back(probs[i].n);
    key.push_back(probs[i].m);
    key.push_back(probs[i].T);
  }
  return key;
}

// Caller holds g_plan_mu.
void retire(std::unique_ptr<Upload>& u) {
  if (u) g_retired.push_back(std::move(u));
}

void release_finished_uploads() {
  for (size_t i = 0; i < g_retired.size();) {
    Upload* u = g_retired[i].get();
    if (!u->done || hipEventQuery(u->done) != hipErrorNotReady) {
      if (u->done) (void)hipEventDestroy(u->done);
      g_retired[i] = std::move(g_retired.back());
      g_retired.pop_back();
    } else {
      ++i;
    }
  }
}

// A call that only writes scratch in the layout of `key` (lqr_solve,
// lqr_solve_phase): plans of another layout in this workspace may be
// overwritten, so they are forgotten (a later capture needs a fresh upload).
void forget_other_layouts(void* ws, const std::vector<int32_t>& key) {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  auto it = g_plans.find(ws);
  if (it == g_plans.end() || it->second.layout == key) return;
  retire(it->second.fwd);
  retire(it->second.adj);
  g_plans.erase(it);
}

// Upload `table` to ws + off (uncaptured stream), or check that exactly this
// plan is resident (captured stream). `adj` selects the plan slot.
lqr_status_t place_plan(void* ws, size_t off, bool adj, const std::vector<int32_t>& key,
                        std::vector<char>&& table, hipStream_t s) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return LQR_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_plan_mu);
  if (cap != hipStreamCaptureStatusNone) {
    auto it = g_plans.find(ws);
    if (it == g_plans.end() || it->second.layout != key) return LQR_ERR_INVALID_ARG;
    const std::unique_ptr<Upload>& u = adj ? it->second.adj : it->second.fwd;
    return (u && u->bytes == table) ? LQR_SUCCESS : LQR_ERR_INVALID_ARG;
  }
  release_finished_uploads();
  WsPlans& w = g_plans[ws];
  if (w.layout != key) {  // another problem set's regions: its plans are overwritten
    retire(w.fwd);
    retire(w.adj);
    w.layout = key;
  }
  std::unique_ptr<Upload>& slot = adj ? w.adj : w.fwd;
  retire(slot);
  std::unique_ptr<Upload> u(new Upload);
  u->bytes = std::move(table);
  if (hipMemcpyAsync(static_cast<char*>(ws) + off, u->bytes.data(), u->bytes.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return LQR_ERR_HIP;
  if (hipEventCreateWithFlags(&u->done, hipEventDisableTiming) != hipSuccess) {
    u->done = nullptr;
    g_retired.push_back(std::move(u));  // kept until the process ends
    return LQR_ERR_HIP;
  }
  if (hipEventRecord(u->done, s) != hipSuccess) {
    (void)hipEventDestroy(u->done);
    u->done = nullptr;
    g_retired.push_back(std::move(u));
    return LQR_ERR_HIP;
  }
  slot = std::move(u);
  return LQR_SUCCESS;
}

}  // namespace

// lqr_solve on a caller-given device buffer (the workspace, or the library's
// own scratch array for lqr_solve_noalloc). Allocates no device memory.
lqr_status_t solve_single(const lqr_problem_t* prob, const lqr_options_t* opts, void* ws,
                          size_t ws_bytes, void* stream) {
  BatchPlan plan;
  lqr_status_t st = make_plan(prob, 1, opts, &plan);
  if (st != LQR_SUCCESS) return st;
  if ((st = check_pointers(*prob)) != LQR_SUCCESS) return st;
  if ((st = check_device(plan)) != LQR_SUCCESS) return st;
  if (!ws || ws_bytes < plan.total_bytes) return LQR_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return LQR_ERR_INVALID_ARG;
  if (is_smoothed(opts) && plan.big) return LQR_ERR_UNSUPPORTED;
  forget_other_layouts(ws, layout_key(prob, 1));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int eng = launch_engine(plan.max_n, is_mixed(opts) || is_f32(opts));
  InstDesc d;
  CvtList cin{}, cout{};
  if (is_f32(opts)) {
    d = make_desc_f32(*prob, plan.inst[0].J, static_cast<char*>(ws), plan.inst[0].ws_off,
                      plan.inst[0].stage_off, cin.it, &cin.n, cout.it, &cout.n);
  } else {
    d = make_desc(*prob, plan.inst[0].J, static_cast<char*>(ws), plan.inst[0].ws_off);
  }
  hipError_t e = launch_convert_list(cin, s);
  if (e == hipSuccess) {
    if (plan.big) {
      const int beng = big_engine(opts);
      if (is_serial(opts)) {
        e = launch_big_sweep(d, 0, beng, plan.lds_serial, s);
      } else {
        e = launch_big_sweep(d, 1, beng, plan.lds1, s);
        if (e == hipSuccess) e = launch_big_link(d, plan.lds2, s);
        if (e == hipSuccess) e = launch_big_sweep(d, 3, beng, plan.lds3, s);
      }
    } else {
      if ((is_serial(opts) || d.J == 1) && small_enough(plan)) {
        // one segment is the plain recursion
        e = launch_small_serial(d, nullptr, 1, s);
      } else if (is_serial(opts)) {
        e = launch_serial(d, plan.lds_serial, eng, s);
      } else if (is_smoothed(opts)) {
        e = launch_phase(d, 1, plan.lds1, eng, s);
        if (e == hipSuccess) e = launch_phase(d, 2, plan.lds2, eng, s);
        if (e == hipSuccess) e = launch_smooth_seed(d, plan.lds2, s);
        if (e == hipSuccess) e = launch_phase(d, 3, plan.lds3, eng, s);
      } else {
        e = launch_parallel(d, plan.lds1, plan.lds2, plan.lds3, eng, s);
      }
    }
  }
  if (e == hipSuccess) e = launch_convert_list(cout, s);
  return e == hipSuccess ? LQR_SUCCESS : LQR_ERR_HIP;
}

// Bytes lqr_solve needs for this problem (the plan's total), or an error.
lqr_status_t solve_bytes(const lqr_problem_t* prob, const lqr_options_t* opts, size_t* bytes) {
  BatchPlan plan;
  lqr_status_t st = make_plan(prob, 1, opts, &plan);
  if (st == LQR_SUCCESS) *bytes = plan.total_bytes;
  return st;
}

}  // namespace lqr

using namespace lqr;

extern "C" {

const char* lqr_status_string(lqr_status_t s) {
  switch (s) {
    case LQR_SUCCESS: return "success";
    case LQR_ERR_INVALID_ARG: return "invalid argument";
    case LQR_ERR_NOT_PD: return "input Hessian not positive definite";
    case LQR_ERR_SINGULAR_COUPLING: return "singular linking system";
    case LQR_ERR_NONFINITE: return "non-finite value";
    case LQR_ERR_WORKSPACE: return "workspace missing or too small";
    case LQR_ERR_HIP: return "HIP runtime error";
    case LQR_ERR_UNSUPPORTED: return "unsupported size or mode";
  }
  return "unknown status";
}

lqr_status_t lqr_workspace_size(const lqr_problem_t* probs, int32_t batch, const lqr_options_t* opts,
                                size_t* bytes) {
  try {
    if (!bytes) return LQR_ERR_INVALID_ARG;
    BatchPlan plan;
    lqr_status_t st = make_plan(probs, batch, opts, &plan);
    if (st != LQR_SUCCESS) return st;
    size_t need = plan.total_bytes;
    AdjPlan ap;  // lqr_backward on the same problems uses the same workspace
    if (make_adj_plan(probs, batch, &ap, is_f32(opts)) == LQR_SUCCESS) need = std::max(need, ap.total_bytes);
    *bytes = need;
    return LQR_SUCCESS;
  } catch (const std::bad_alloc&) {
    return LQR_ERR_INVALID_ARG;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_workspace_layout(const lqr_problem_t* probs, int32_t batch,
                                  const lqr_options_t* opts, size_t* out) {
  try {
    if (!out) return LQR_ERR_INVALID_ARG;
    BatchPlan plan;
    lqr_status_t st = make_plan(probs, batch, opts, &plan);
    if (st != LQR_SUCCESS) return st;
    AdjPlan ap;
    const bool adj_ok = make_adj_plan(probs, batch, &ap, is_f32(opts)) == LQR_SUCCESS;
    out[0] = 0;
    out[1] = plan.reg.adj_cap;
    out[2] = plan.reg.fwd_off;
    out[3] = plan.reg.fwd_cap;
    out[4] = plan.reg.scratch_off;
    out[5] = adj_ok ? ap.table_bytes : 0;
    out[6] = plan.table_bytes;
    out[7] = adj_ok ? std::max(plan.total_bytes, ap.total_bytes) : plan.total_bytes;
    return LQR_SUCCESS;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_solve(const lqr_problem_t* prob, const lqr_options_t* opts, void* ws,
                       size_t ws_bytes, void* stream) {
  try {
    return lqr::solve_single(prob, opts, ws, ws_bytes, stream);
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_solve_phase(const lqr_problem_t* prob, const lqr_options_t* opts, int32_t phase,
                             void* ws, size_t ws_bytes, void* stream) {
  try {
    if (phase < 1 || phase > 3) return LQR_ERR_INVALID_ARG;
    if (is_f32(opts)) return LQR_ERR_UNSUPPORTED;  // phases work on FP64 arrays in place
    BatchPlan plan;
    lqr_status_t st = make_plan(prob, 1, opts, &plan);
    if (st != LQR_SUCCESS) return st;
    if (is_smoothed(opts) && plan.big) return LQR_ERR_UNSUPPORTED;
    if ((st = check_pointers(*prob)) != LQR_SUCCESS) return st;
    if ((st = check_device(plan)) != LQR_SUCCESS) return st;
    if (!ws || ws_bytes < plan.total_bytes) return LQR_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return LQR_ERR_INVALID_ARG;
    forget_other_layouts(ws, layout_key(prob, 1));
    const InstDesc d = make_desc(*prob, plan.inst[0].J, static_cast<char*>(ws), plan.inst[0].ws_off);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    const int eng = launch_engine(plan.max_n, is_mixed(opts));
    if (plan.big) {
      const int beng = big_engine(opts);
      if (is_serial(opts)) {
        if (phase == 1) e = launch_big_sweep(d, 0, beng, plan.lds_serial, s);
      } else if (phase == 2) {
        e = launch_big_link(d, plan.lds2, s);
      } else {
        e = launch_big_sweep(d, phase, beng, phase == 1 ? plan.lds1 : plan.lds3, s);
      }
    } else if (is_serial(opts)) {
      if (phase == 1)
        e = small_enough(plan) ? launch_small_serial(d, nullptr, 1, s)
                               : launch_serial(d, plan.lds_serial, eng, s);
    } else {
      const size_t lds = phase == 1 ? plan.lds1 : phase == 2 ? plan.lds2 : plan.lds3;
      e = launch_phase(d, phase, lds, eng, s);
      if (e == hipSuccess && phase == 2 && is_smoothed(opts)) e = launch_smooth_seed(d, plan.lds2, s);
    }
    return e == hipSuccess ? LQR_SUCCESS : LQR_ERR_HIP;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_link_multipliers(const lqr_problem_t* prob, const lqr_options_t* opts,
                                  int32_t segments, void* mu, void* stream) {
  try {
    if (!prob) return LQR_ERR_INVALID_ARG;
    lqr_status_t st = check_options(opts);
    if (st != LQR_SUCCESS) return st;
    if ((st = check_dims(*prob)) != LQR_SUCCESS) return st;
    if (segments < 1 || segments > prob->T || prob->n > lqr::kBigMaxN) return LQR_ERR_INVALID_ARG;
    if (segments == 1) return LQR_SUCCESS;
    if (!prob->P || !prob->p || !prob->x || !mu) return LQR_ERR_INVALID_ARG;
    const hipError_t e = lqr::launch_link_mu(prob->n, prob->T, segments, prob->P, prob->p, prob->x, mu,
                                        is_f32(opts), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LQR_SUCCESS : LQR_ERR_HIP;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_plan_segments(const lqr_problem_t* probs, int32_t batch, const lqr_options_t* opts,
                               int32_t* segments, double* est_us) {
  try {
    if (!segments) return LQR_ERR_INVALID_ARG;
    BatchPlan plan;
    lqr_status_t st = make_plan(probs, batch, opts, &plan);
    if (st != LQR_SUCCESS) return st;
    for (int i = 0; i < batch; ++i) segments[i] = plan.inst[i].J;
    if (est_us) *est_us = plan.est_us;
    return LQR_SUCCESS;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_solve_batched(const lqr_problem_t* probs, int32_t batch, const lqr_options_t* opts,
                               void* ws, size_t ws_bytes, void* stream) {
  try {
    if (is_smoothed(opts) && check_options(opts) == LQR_SUCCESS) return LQR_ERR_UNSUPPORTED;
    BatchPlan plan;
    lqr_status_t st = make_plan(probs, batch, opts, &plan);
    if (st != LQR_SUCCESS) return st;
    // a large-state instance (batch of one): the single-instance launches
    if (plan.big) return solve_single(probs, opts, ws, ws_bytes, stream);
    for (int i = 0; i < batch; ++i)
      if ((st = check_pointers(probs[i])) != LQR_SUCCESS) return st;
    if ((st = check_device(plan)) != LQR_SUCCESS) return st;
    if (!ws || ws_bytes < plan.total_bytes) return LQR_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return LQR_ERR_INVALID_ARG;
    char* base = static_cast<char*>(ws);
    const bool serial = is_serial(opts);

    // Host image of the plan: descriptors; (instance, segment) items of the
    // phased launches, longest segments first; the persistent task order.
    std::vector<char> table(plan.table_bytes, 0);
    InstDesc* descs = reinterpret_cast<InstDesc*>(table.data());
    WorkItem* items = reinterpret_cast<WorkItem*>(table.data() + (plan.items_off - plan.table_off));
    TaskItem* tasks = reinterpret_cast<TaskItem*>(table.data() + (plan.tasks_off - plan.table_off));
    const bool f32 = is_f32(opts);
    CvtItem* cvt = reinterpret_cast<CvtItem*>(table.data() + (plan.cvt_off - plan.table_off));
    std::vector<CvtItem> couts;
    int ncin = 0;
    std::vector<std::pair<double, WorkItem>> order;
    order.reserve(plan.nitems);
    for (int i = 0; i < batch; ++i) {
      if (f32) {
        CvtItem ci[kMaxCvt], co[kMaxCvt];
        int ni = 0, no = 0;
        descs[i] = make_desc_f32(probs[i], plan.inst[i].J, base, plan.inst[i].ws_off,
                                 plan.inst[i].stage_off, ci, &ni, co, &no);
        for (int k = 0; k < ni; ++k) cvt[ncin++] = ci[k];
        couts.insert(couts.end(), co, co + no);
      } else {
        descs[i] = make_desc(probs[i], plan.inst[i].J, base, plan.inst[i].ws_off);
      }
      const lqr_problem_t& p = probs[i];
      const int J = plan.inst[i].J;
      for (int j = 0; j < J; ++j) {
        const int len = seg_begin(p.T, J, j + 1) - seg_begin(p.T, J, j);
        const double cost = (double)len * (double)p.n * p.n * (p.n + p.m);
        order.push_back({cost, WorkItem{i, j}});
      }
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, WorkItem>& a, const std::pair<double, WorkItem>& b) {
                       return a.first > b.first;
                     });
    for (int i = 0; i < plan.nitems; ++i) items[i] = order[i].second;
    std::copy(plan.tasks.begin(), plan.tasks.end(), tasks);
    std::copy(couts.begin(), couts.end(), cvt + ncin);
    const int ncout = (int)couts.size();

    hipStream_t s = static_cast<hipStream_t>(stream);
    st = place_plan(ws, plan.table_off, false, layout_key(probs, batch), std::move(table), s);
    if (st != LQR_SUCCESS) return st;
    const InstDesc* ddesc = reinterpret_cast<const InstDesc*>(base + plan.table_off);
    const WorkItem* ditems = reinterpret_cast<const WorkItem*>(base + plan.items_off);
    const TaskItem* dtasks = reinterpret_cast<const TaskItem*>(base + plan.tasks_off);
    int32_t* dsync = reinterpret_cast<int32_t*>(base + plan.sync_off);
    const CvtItem* dcvt = reinterpret_cast<const CvtItem*>(base + plan.cvt_off);
    hipError_t e = launch_convert(dcvt, ncin, s);
    if (e != hipSuccess) return LQR_ERR_HIP;
    const int eng = launch_engine(plan.max_n, is_mixed(opts) || f32);
    // With one segment per instance the parallel algorithm is the plain
    // recursion; one workgroup per instance runs it without the task queue.
    bool single = true;
    for (int i = 0; i < batch && single; ++i) single = plan.inst[i].J == 1;
    if ((serial || (single && !is_phased(opts))) && small_enough(plan))
      e = launch_small_serial(InstDesc{}, ddesc, batch, s);
    else if (serial || (single && !is_phased(opts)))
      e = launch_serial_batched(ddesc, batch, plan.max_m, eng, plan.lds_serial, s);
    else if (is_phased(opts))
      e = launch_parallel_batched(ddesc, ditems, plan.nitems, batch, plan.max_n, plan.max_m,
                                  plan.lds1, plan.lds2, plan.lds3, eng, s);
    else
      e = launch_persistent(ddesc, dtasks, (int)plan.tasks.size(), batch, dsync,
                            kernel_width(plan.max_m, eng), eng,
                            plan.lds_persist, nullptr, s);
    if (e == hipSuccess) e = launch_convert(dcvt + ncin, ncout, s);
    return e == hipSuccess ? LQR_SUCCESS : LQR_ERR_HIP;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

lqr_status_t lqr_backward(const lqr_problem_t* probs, int32_t batch, const lqr_grad_t* grads,
                          const lqr_options_t* opts, void* ws, size_t ws_bytes, void* stream) {
  try {
    lqr_status_t st = check_options(opts);
    if (st != LQR_SUCCESS) return st;
    if (is_smoothed(opts)) return LQR_ERR_UNSUPPORTED;
    if (!grads) return LQR_ERR_INVALID_ARG;
    AdjPlan ap;
    const bool f32 = is_f32(opts);
    if ((st = make_adj_plan(probs, batch, &ap, f32)) != LQR_SUCCESS) return st;
    for (int i = 0; i < batch; ++i) {
      const lqr_problem_t& p = probs[i];
      if (!p.A || !p.B || !p.K || !p.P || !p.x || !p.u || !p.lam || !p.chol) return LQR_ERR_INVALID_ARG;
      if (!grads[i].dl_dx || !grads[i].dl_du) return LQR_ERR_INVALID_ARG;
    }
    if (!ws || ws_bytes < ap.total_bytes) return LQR_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return LQR_ERR_INVALID_ARG;
    char* base = static_cast<char*>(ws);
    std::vector<char> table(ap.table_bytes, 0);
    AdjDesc* descs = reinterpret_cast<AdjDesc*>(table.data());
    int2* blocks = reinterpret_cast<int2*>(table.data() + ap.blocks_off);
    CvtItem* cvt = reinterpret_cast<CvtItem*>(table.data() + ap.cvt_off);
    std::vector<CvtItem> couts;
    int ncin = 0;
    int nb = 0;
    for (int i = 0; i < batch; ++i) {
      const lqr_problem_t& p = probs[i];
      const lqr_grad_t& g = grads[i];
      AdjDesc& a = descs[i];
      a.n = p.n; a.m = p.m; a.T = p.T; a.pad_ = 0;
      a.A = static_cast<const double*>(p.A);
      a.B = static_cast<const double*>(p.B);
      a.K = static_cast<const double*>(p.K);
      a.P = static_cast<const double*>(p.P);
      a.chol = static_cast<const double*>(p.chol);
      a.x = static_cast<const double*>(p.x);
      a.u = static_cast<const double*>(p.u);
      a.lam = static_cast<const double*>(p.lam);
      a.dl_dx = static_cast<const double*>(g.dl_dx);
      a.dl_du = static_cast<const double*>(g.dl_du);
      a.dA = static_cast<double*>(g.dA);
      a.dB = static_cast<double*>(g.dB);
      a.dc = static_cast<double*>(g.dc);
      a.dQ = static_cast<double*>(g.dQ);
      a.dq = static_cast<double*>(g.dq);
      a.dR = static_cast<double*>(g.dR);
      a.dr = static_cast<double*>(g.dr);
      a.dS = static_cast<double*>(g.dS);
      a.dx0 = static_cast<double*>(g.dx0);
      a.ws = reinterpret_cast<double*>(base + ap.ws_off[i]);
      if (f32) {  // FP64 staging of every array the adjoint reads or writes
        const size_t t = p.T, t1 = (size_t)p.T + 1, n = p.n, m = p.m;
        double* q = reinterpret_cast<double*>(base + ap.stage_off[i]);
        auto in = [&](const void* user, size_t count) -> const double* {
          double* dst = q;
          q += count;
          if (!user) return nullptr;
          cvt[ncin++] = CvtItem{user, dst, (int64_t)count, 1, 0};
          return dst;
        };
        auto out = [&](void* user, size_t count) -> double* {
          double* src = q;
          q += count;
          if (!user) return nullptr;
          couts.push_back(CvtItem{src, user, (int64_t)count, 0, 0});
          return src;
        };
        a.A = in(p.A, t * n * n);
        a.B = in(p.B, t * n * m);
        a.K = in(p.K, t * m * n);
        a.P = in(p.P, t1 * n * n);
        a.chol = in(p.chol, t * m * m);
        a.x = in(p.x, t1 * n);
        a.u = in(p.u, t * m);
        a.lam = in(p.lam, t1 * n);
        a.dl_dx = in(g.dl_dx, t1 * n);
        a.dl_du = in(g.dl_du, t * m);
        a.dA = out(g.dA, t * n * n);
        a.dB = out(g.dB, t * n * m);
        a.dc = out(g.dc, t * n);
        a.dQ = out(g.dQ, t1 * n * n);
        a.dq = out(g.dq, t1 * n);
        a.dR = out(g.dR, t * m * m);
        a.dr = out(g.dr, t * m);
        a.dS = out(g.dS, t * m * n);
        a.dx0 = out(g.dx0, n);
      }
      const int nbi = (p.T + 1 + kAdjStages - 1) / kAdjStages;
      for (int b = 0; b < nbi; ++b) blocks[nb++] = int2{i, b};
    }
    std::copy(couts.begin(), couts.end(), cvt + ncin);
    const int ncout = (int)couts.size();
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = place_plan(ws, 0, true, layout_key(probs, batch), std::move(table), s);
    if (st != LQR_SUCCESS) return st;
    const CvtItem* dcvt = reinterpret_cast<const CvtItem*>(base + ap.cvt_off);
    hipError_t e = launch_convert(dcvt, ncin, s);
    if (e == hipSuccess)
      e = launch_adjoint(reinterpret_cast<const AdjDesc*>(base), batch,
                         reinterpret_cast<const int2*>(base + ap.blocks_off), nb, ap.lds, s);
    if (e == hipSuccess) e = launch_convert(dcvt + ncin, ncout, s);
    return e == hipSuccess ? LQR_SUCCESS : LQR_ERR_HIP;
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}

}  // extern "C"
