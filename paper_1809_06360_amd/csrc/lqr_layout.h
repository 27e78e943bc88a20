// Shapes shared by the host planner and the kernels: the per-instance device
// descriptor, segment boundaries, workspace strides and LDS footprints.
#pragma once

#include <stddef.h>
#include <stdint.h>

#ifndef LQR_HD
#if defined(__HIPCC__)
#define LQR_HD __host__ __device__ inline
#else
#define LQR_HD inline
#endif
#endif

namespace lqr {

// One instance as the kernels see it (FP64 element type). Built on the host
// from lqr_problem_t plus the workspace carve-out; passed by value to the
// single-instance kernels and stored in a device table for batched launches.
struct InstDesc {
  int32_t n, m, T, J;
  const double *A, *B, *c, *Q, *q, *R, *r, *S, *x0;
  double *K, *k, *P, *p, *x, *u, *lam, *chol;
  int32_t *info;
  double *ws;      // per-instance scratch (segment summaries, boundary values, link maps)
  int32_t *fail;   // [J] first failing stage + 1 seen by each segment's sweep, 0 if none
};

// One instance of the adjoint (gradient) computation: forward data and
// outputs, upstream gradients, gradient outputs (nullptr = not written) and
// a per-instance scratch area (phat, khat, xhat, uhat, lamhat).
struct AdjDesc {
  int32_t n, m, T, pad_;
  const double *A, *B, *K, *P, *chol, *x, *u, *lam;
  const double *dl_dx, *dl_du;
  double *dA, *dB, *dc, *dQ, *dq, *dR, *dr, *dS, *dx0;
  double* ws;
};

// Stages per workgroup of the gradient outer-product kernel.
constexpr int kAdjStages = 8;

LQR_HD size_t adj_ws_doubles(int n, int m, int T) {
  return 3 * (size_t)(T + 1) * n + 2 * (size_t)T * m;
}
LQR_HD size_t adj_lds(int n, int m) {
  return (3 * (size_t)n + 3 * (size_t)m + (size_t)m * m) * 8 + 64;
}

// A unit of batched work: instance index and segment index.
struct WorkItem {
  int32_t inst, seg;
};

// One array conversion between the caller's FP32 buffers and the FP64 staging
// area of the FP32 precision mode (count elements; to_f64: float -> double,
// else double -> float).
struct CvtItem {
  const void* src;
  void* dst;
  int64_t count;
  int32_t to_f64;
  int32_t pad_;
};

// Conversions of one instance, passed by value to single-instance launches:
// at most 9 inputs (A, B, c, Q, q, R, r, S, x0) or 8 outputs.
constexpr int kMaxCvt = 9;
struct CvtList {
  CvtItem it[kMaxCvt];
  int32_t n;
};

// FP64 staging of one instance in the FP32 mode: inputs
// A | B | c | Q | q | R | r | S | x0, then outputs K | k | P | p | x | u | lam | chol.
LQR_HD size_t stage_in_doubles(int n, int m, int T) {
  return (size_t)T * n * n + (size_t)T * n * m + (size_t)T * n + (size_t)(T + 1) * n * n +
         (size_t)(T + 1) * n + (size_t)T * m * m + (size_t)T * m + (size_t)T * m * n + n;
}
LQR_HD size_t stage_out_doubles(int n, int m, int T) {
  return (size_t)T * m * n + (size_t)T * m + (size_t)(T + 1) * n * n + 3 * (size_t)(T + 1) * n +
         (size_t)T * m + (size_t)T * m * m;
}

// A task of the persistent batched launch: phase 1 (segment sweep), 2
// (linking solve, seg unused) or 3 (rebuild and forward simulation) of one
// (instance, segment). Tasks are taken from a queue in table order, which the
// host makes a topological order of the dependencies
//   every phase-1 task of an instance  ->  its phase-2 task  ->  its phase-3 tasks.
struct TaskItem {
  int32_t inst, seg, phase;
};

// Synchronisation words of a persistent launch (int32, zeroed before every
// launch): the queue head, then per instance the number of finished phase-1
// tasks, then per instance the finished flag of its phase-2 task.
LQR_HD size_t sync_words(int ninst) { return 64 + 2 * (size_t)ninst; }
constexpr int kSyncHead = 0;
constexpr int kSyncDone1 = 64;  // the head sits alone in its 256-byte line

// Segment j covers stages [seg_begin(j), seg_begin(j+1)); the first T mod J
// segments are one stage longer.
LQR_HD int seg_begin(int T, int J, int j) {
  const int L = T / J, extra = T % J;
  return j * L + (j < extra ? j : extra);
}

// Workspace strides, in doubles.
//  seg[j], j < J-1 : P0 (n*n) | Gamma (n*n) | Psi (n*n) | pbar (n) | psi (n)
//  bnd[j], j < J   : P (n*n) | p (n) | x (n)           value and state at seg_begin(j)
//  link[j], j < J-1: F (n*n, column-major) | f (n)     x_{t_{j+1}} = F x_{t_j} + f
//                    (column-major so that the serial forward chain, lane i
//                    taking row i, reads each column with one coalesced load)
LQR_HD size_t seg_stride(int n) { return 3 * (size_t)n * n + 2 * (size_t)n; }
LQR_HD size_t bnd_stride(int n) { return (size_t)n * n + 2 * (size_t)n; }
LQR_HD size_t link_stride(int n) { return (size_t)n * n + (size_t)n; }

//  scan[w][j], w = 0, 1, j < J: two buffers of J summaries (seg layout) for
//                    the logarithmic-depth linking solve
LQR_HD size_t ws_doubles(int n, int J) {
  return (size_t)(J - 1) * seg_stride(n) + (size_t)J * bnd_stride(n) +
         (size_t)(J - 1) * link_stride(n) + 2 * (size_t)J * seg_stride(n);
}
LQR_HD double* ws_seg(double* ws, int n, int j) { return ws + (size_t)j * seg_stride(n); }
LQR_HD double* ws_bnd(double* ws, int n, int J, int j) {
  return ws + (size_t)(J - 1) * seg_stride(n) + (size_t)j * bnd_stride(n);
}
LQR_HD double* ws_link(double* ws, int n, int J, int j) {
  return ws + (size_t)(J - 1) * seg_stride(n) + (size_t)J * bnd_stride(n) +
         (size_t)j * link_stride(n);
}

LQR_HD double* ws_scan(double* ws, int n, int J, int w) {
  return ws + (size_t)(J - 1) * seg_stride(n) + (size_t)J * bnd_stride(n) +
         (size_t)(J - 1) * link_stride(n) + (size_t)w * J * seg_stride(n);
}

// Int32 words per instance after the scratch: J per-segment stage-failure
// words, then the linking-failure word.
LQR_HD size_t fail_words(int J) { return (size_t)J + 1; }

// The single-instance linking solve runs in logarithmic depth (scan of the
// segment summaries) from this many segments on, and serially below.
constexpr int kTreeMinJ = 8;
LQR_HD bool use_link_tree(int n, int J) { return J >= kTreeMinJ && n <= 64; }

// LDS footprints in bytes (FP64). The sweep keeps, per workgroup:
//  sP  n x n           value Hessian of the next stage
//  sp  n               value gradient
//  sX  n x (m+n+1)     [B_t | A_t | c_t]
//  sY  n x W           [P B | P A | P c + p | Gamma]          (Gamma: dual sweep only)
//  sG  mp x W          [R + B'PB | S + B'PA | r + B'(Pc+p) | B'Gamma], column-major
//                      with leading dimension mp = pad_rows(m) + 1
//  dual only: sPsi n x n, spsi n, sgc n
//                      (after the elimination its first m columns hold L^{-1})
//  sE  3 pad_rows(m)   elimination exchange vectors and pivots
//  dual only: sPsi n x n, spsi n, sgc n
// with W = m + n + 1 (+ n for the dual sweep).
LQR_HD int sweep_w(int n, int m, bool dual) { return m + n + 1 + (dual ? n : 0); }

// Column-owner elimination of the input Hessian (see ldl_columns): one thread
// per column of [H | right-hand sides (| identity)], at most 256 columns, and
// m <= 64 rows held in registers.
LQR_HD bool sweep_fits_regs(int n, int m, bool dual) {
  const int cols = dual ? m + 2 * n + 1 : 2 * m + n + 1;
  return m <= 64 && cols <= 256;
}

LQR_HD int pad_rows(int m) { return m <= 8 ? 8 : m <= 16 ? 16 : m <= 24 ? 24 : m <= 32 ? 32 : m <= 48 ? 48 : 64; }

// `mw` is the register width of the kernel variant that runs the sweep
// (pad_rows of the largest m in the launch).
// Leading dimension of the value Hessian P in a sweep's LDS: n rounded up to
// an odd count.
LQR_HD int p_ld(int n) { return n | 1; }

LQR_HD size_t sweep_lds(int n, int m, bool dual, int mw) {
  const size_t W = (size_t)sweep_w(n, m, dual), mp = (size_t)mw + 1;
  size_t dbl = (size_t)n * p_ld(n) + n + (size_t)n * (m + n + 1) + (size_t)n * W + mp * W +
               3 * (size_t)mw;
  if (dual) dbl += (size_t)n * n + 2 * (size_t)n;
  return dbl * 8 + 64;
}

// LDS a workgroup may hold on gfx950; a segment sweep whose resident layout
// needs more runs its streamed form (see dual_sweep_gs).
constexpr size_t kLdsSweepMax = 160 * 1024;

// LDS of the streamed parametric sweep: P, p, [B | c], P[B | A | c] + [0|0|p],
// the Hessian block (mw+1) x (m+2n+1), exchange vectors, psi and Gam'c
// (Gamma and Psi stay in global memory).
LQR_HD size_t sweep_lds_gs(int n, int m, int mw) {
  const size_t W = (size_t)m + 2 * (size_t)n + 1, mp = (size_t)mw + 1;
  const size_t dbl = (size_t)n * p_ld(n) + n + (size_t)n * (m + 1) + (size_t)n * (m + n + 1) + mp * W +
                     3 * (size_t)mw + 2 * (size_t)n;
  return dbl * 8 + 64;
}

// LDS the parametric sweep of phase 1 uses: the resident layout if it fits,
// else the streamed one.
LQR_HD size_t dual_lds(int n, int m, int mw) {
  const size_t r = sweep_lds(n, m, true, mw);
  return r <= kLdsSweepMax ? r : sweep_lds_gs(n, m, mw);
}

// Problems with at least this many states run their products on matrix cores.
constexpr int kMfmaMinN = 32;

// LDS of the serial linking solve (defined below).
LQR_HD size_t couple_lds(int n, int nw);

// Register width of the linking solve inside the persistent kernel: one
// width per product engine (MFMA variants serve n <= 64, VALU ones n < 32).
LQR_HD constexpr int persist_nw(bool mf) { return mf ? 64 : 32; }

// Doubles of LDS for the workgroup inversion's exchange (wg_invert): two
// slots of 64 multipliers, two reciprocal pivots, two pivot rows and a flag.
constexpr int kInvExchangeDoubles = 132;

// Leading dimension of an n x n block in LDS: odd, so that the 16 lanes of a
// matrix-core operand fragment that walk a strided row or column of the block
// hit distinct LDS banks.
LQR_HD constexpr int ld_odd(int n) { return n | 1; }

// Join of two summaries: the four n x n operands staged in LDS (register
// widths up to 48; wider joins read them from global memory), four n x n
// work blocks (M and its inverse, the right-hand side, and two products of
// the inverse), four vectors and the inversion's exchange.
LQR_HD constexpr bool link_tree_staged(int nw) { return nw <= 48; }

LQR_HD size_t link_tree_lds(int n, int nw) {
  const size_t blk = (size_t)n * ld_odd(n);
  const size_t dbl = (link_tree_staged(nw) ? 8 : 4) * blk + 4 * (size_t)n + kInvExchangeDoubles;
  return dbl * 8 + 64;
}

// Forward chain over the boundaries: double-buffered chunks of S link maps
// (link_stride(n) doubles each) and of their S boundary states (64 doubles
// each), within about 150 KiB, and the state vector.
LQR_HD int link_forward_slots(int n) {
  const size_t per = (size_t)n * n + n + 64;
  const size_t s = (150u * 1024u / 8u - 64u) / (2 * per);
  return s < 1 ? 1 : (s > 16 ? 16 : (int)s);
}
LQR_HD size_t link_forward_lds(int n) {
  return (64 + 2 * (size_t)link_forward_slots(n) * ((size_t)n * n + n + 64)) * 8;
}

// ---------------------------------------------------------------------------
// Large-state path (65..128 states, up to 64 inputs; 256-thread sweep and
// 512-thread linking workgroups).
// ---------------------------------------------------------------------------
constexpr int kBigMaxN = 128;
constexpr int kBigMaxM = 64;
LQR_HD bool is_big(int n, int m) { return n > 64 && n <= kBigMaxN && m <= kBigMaxM; }

// Sweep scratch of one segment, in doubles (sized for double elements; the
// FP32-product engine stores float and uses half): P (n x n) | Y = P[B | A | c]
// (n x (m+n+1)) | Gamma, twice (n x n each) | Psi (n x n) | right-hand sides
// and their eliminated form Z (m x (2n+1) each).
LQR_HD size_t big_sweep_doubles(int n, int m) {
  const size_t nn = (size_t)n * n;
  return nn + (size_t)n * (m + n + 1) + 2 * nn + nn + 2 * (size_t)m * (2 * n + 1);
}
// Join scratch of one scan element: four n x n products and the inverted
// linking matrix.
LQR_HD size_t big_join_doubles(int n) { return 5 * (size_t)n * n; }
// Per-instance workspace of the large-state path: that of ws_doubles, then J
// sweep scratches, then J join scratches.
LQR_HD size_t big_ws_doubles(int n, int m, int J) {
  return ws_doubles(n, J) + (size_t)J * (big_sweep_doubles(n, m) + big_join_doubles(n));
}
LQR_HD double* big_sweep_ws(double* ws, int n, int m, int J, int seg) {
  return ws + ws_doubles(n, J) + (size_t)seg * big_sweep_doubles(n, m);
}
LQR_HD double* big_join_ws(double* ws, int n, int m, int J, int j) {
  return ws + ws_doubles(n, J) + (size_t)J * big_sweep_doubles(n, m) + (size_t)j * big_join_doubles(n);
}
// LDS of the large-state kernels: first the two panel buffers of their
// matrix-core products (kBigPanelBytes), then for the sweeps the input Hessian
// and L^{-1} (m x 65 doubles each, column-major), the elimination's exchange
// vector, five n-vectors and flag words (the forward simulation reuses the
// start: x, u); for the linking kernels the inverse's exchange space, four
// n-vectors and the pivot maps.
constexpr size_t kBigPanelBytes = 68608;
LQR_HD size_t big_sweep_lds() { return kBigPanelBytes + (2 * 64 * 65 + 3 * 64 + 5 * 128) * 8 + 64; }
LQR_HD size_t big_link_lds() { return kBigPanelBytes + (512 + 4 * 128) * 8 + 256 * 4 + 64; }

// Partial sums of the forward simulation's matrix-vector products (n, m <= 64)
// and one flag word per wave.
LQR_HD size_t rollout_lds(int /*n*/, int /*m*/) { return (4 * 128 + 4 * 64) * 8 + 64; }

// `nw` is the register width of the kernel variant (pad_rows of the largest n).
// Four n x n blocks (exact value, Psi then Gam, N then its inverse, F), five
// vectors, the inversion's exchange and two flag words.
LQR_HD size_t couple_lds(int n, int /*nw*/) {
  const size_t dbl = 4 * (size_t)n * ld_odd(n) + 5 * (size_t)n + kInvExchangeDoubles;
  return dbl * 8 + 4 * 4 + 64;
}

}  // namespace lqr
