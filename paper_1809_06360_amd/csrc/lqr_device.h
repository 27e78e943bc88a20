// Device code of the parallel Riccati recursion (FP64), gfx950.
//
// The horizon [0, T) is cut into J segments (Sec. II-A: dividing into
// sub-trajectories). The three launches are
//   phase 1  one workgroup per segment. Segments j < J-1 run a parametric
//            backward sweep: the segment's optimal cost as a function of its
//            start state AND of a free linear price mu on its end state (the
//            dual form of the endpoint-constrained subproblem (opt:split); mu
//            is the multiplier of the endpoint constraint, eq. term1). The
//            last segment, which carries the terminal cost, runs the plain
//            recursion and is final.
//   phase 2  one workgroup per instance: the linking system (link equation of
//            Sec. II-A and its J-segment generalisation) solved by block
//            elimination from the last boundary backwards; its pivots are the
//            exact value functions at the segment boundaries, and a forward
//            pass gives the exact states at the boundaries (the link points).
//   phase 3  one workgroup per segment: the plain recursion from the exact
//            boundary value rebuilds the segment's gains and value functions,
//            then the segment's trajectory is simulated forward from its exact
//            link point (eq. xopt/uopt evaluated at the link points).
// The serial kernel runs the plain recursion over the whole horizon in one
// workgroup and is the GPU baseline.
#pragma once

#include <hip/hip_runtime.h>

#include "lqr_layout.h"
#include "mi355lqr.h"
#include "wg_linalg.h"

namespace lqr {


// LDS of one sweep. G (input Hessian and right-hand sides) is column-major
// with leading dimension mp = MW + 1 (MW the kernel's register width, >= m):
// element (i, j) at G[j * mp + i]. P is row-major with the odd leading
// dimension ldp = p_ld(n), so that the 16 rows a matrix-core operand fetch
// reads fall in distinct LDS banks.
struct SweepLds {
  double *P, *p, *X, *Y, *G, *E, *Psi, *psi, *gc;
  int* bad;
  int WX, W, mp, ldp;
};

LQR_DEV SweepLds carve_sweep(double* smem, int n, int m, bool dual, int mw) {
  SweepLds s;
  s.WX = m + n + 1;
  s.W = sweep_w(n, m, dual);
  double* q = smem;
  s.ldp = p_ld(n);
  s.P = q; q += n * s.ldp;
  s.p = q; q += n;
  s.X = q; q += n * s.WX;
  s.Y = q; q += n * s.W;
  s.mp = mw + 1;
  s.G = q; q += s.mp * s.W;
  s.E = q; q += 3 * mw;
  s.Psi = s.psi = s.gc = nullptr;
  if (dual) {
    s.Psi = q; q += n * n;
    s.psi = q; q += n;
    s.gc = q; q += n;
  }
  s.bad = reinterpret_cast<int*>(q);
  return s;
}

// Status codes of a sweep (the per-instance info word's encoding): t + 1 for
// the largest stage t whose input Hessian was not positive definite,
// LQR_INFO_NONFINITE if a non-finite value reached a pivot (and no stage was
// found indefinite first), else 0. `bad` is the elimination's flag of stage t
// (1: indefinite, 2: non-finite pivot).
LQR_DEV int note_pivot(int code, int bad, int t) {
  if (bad == 1 && code <= 0) return t + 1;
  if (bad == 2 && code == 0) return LQR_INFO_NONFINITE;
  return code;
}

// Two status codes into one: a stage or linking failure (positive) outranks a
// non-finite value (negative), which outranks success; among positive codes
// the larger wins. Commutative and associative, so the result does not depend
// on the order in which segments report.
LQR_HD int combine_info(int a, int b) { return (a > 0 || b > 0) ? (a > b ? a : b) : (a < b ? a : b); }

// Fold a status code into the instance's info word from concurrent segments.
LQR_DEV void report_info(int32_t* info, int code) {
  if (code > 0)
    atomicMax(info, code);
  else if (code < 0)
    atomicCAS(info, 0, code);
}

// Cache warming for the next stage of a backward sweep: one double of every
// 128-byte line of stage t's inputs (A, B, c, Q, q, R, r, S), up to
// kTouch * kThreads lines, is loaded into registers. Issued right after a
// stage's own inputs are staged, the loads complete while that stage
// computes; sink() stores their sum to a dead LDS word at the end of the
// stage, so the wait for them lands where nothing is pending.
constexpr int kTouch = 6;
struct Touch {
  double v[kTouch];
};

LQR_DEV Touch touch_stage(const InstDesc& d, int t) {
  const int n = d.n, m = d.m;
  const double* base[8] = {d.A + (size_t)t * n * n, d.B + (size_t)t * n * m, d.c + (size_t)t * n,
                           d.Q + (size_t)t * n * n, d.q + (size_t)t * n,     d.R + (size_t)t * m * m,
                           d.r + (size_t)t * m,     d.S ? d.S + (size_t)t * m * n : d.r};
  const int cnt[8] = {n * n, n * m, n, n * n, n, m * m, m, d.S ? m * n : 0};
  Touch h;
#pragma unroll
  for (int k = 0; k < kTouch; ++k) {
    int g = threadIdx.x + k * kThreads;  // line index over the concatenated arrays
    const double* p = nullptr;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int lines = (cnt[a] + 15) >> 4;
      if (!p && g < lines) p = base[a] + 16 * g;
      if (!p) g -= lines;
    }
    h.v[k] = p ? *gp(p) : 0.0;
  }
  return h;
}

LQR_DEV void sink(const Touch& h, double* dead) {
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < kTouch; ++k) a += h.v[k];
  *dead = a;
}

// sum_k M[k * ldm + i] v[k * ldv] for k < n: four independent partial sums,
// so that the loads of several k are in flight at once.
LQR_DEV double col_dot(const double* M, int ldm, const double* v, int ldv, int i, int n) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    a0 = fma(M[k * ldm + i], v[k * ldv], a0);
    a1 = fma(M[(k + 1) * ldm + i], v[(k + 1) * ldv], a1);
    a2 = fma(M[(k + 2) * ldm + i], v[(k + 2) * ldv], a2);
    a3 = fma(M[(k + 3) * ldm + i], v[(k + 3) * ldv], a3);
  }
  for (; k < n; ++k) a0 = fma(M[k * ldm + i], v[k * ldv], a0);
  return (a0 + a1) + (a2 + a3);
}

// Stage inputs into LDS: X = [B_t | A_t | c_t].
LQR_DEV void load_stage(const InstDesc& d, int t, const SweepLds& s) {
  const int n = d.n, m = d.m;
  load_block(s.X, s.WX, d.B + (size_t)t * n * m, m, n, m);
  load_block(s.X + m, s.WX, d.A + (size_t)t * n * n, n, n, n);
  const LQR_GLOBAL double* ct = gp(d.c + (size_t)t * n);
  for (int i = threadIdx.x; i < n; i += kThreads) s.X[i * s.WX + m + n] = ct[i];
}

// Y[:, 0:WX] = P [B | A | c] + [0 | 0 | p]
template <int MM, int E>
LQR_DEV void stage_products(const InstDesc& d, const SweepLds& s) {
  const int n = d.n, m = d.m, WX = s.WX, W = s.W;
  double* Y = s.Y;
  const double* p = s.p;
  pgemm_sub<E, false, false, false, false>(n, WX, n, s.P, s.ldp, s.X, WX, 0, s.P, s.ldp, s.X, WX,
                                        [=](int i, int j, double v) {
                                          if (j == m + n) v += p[i];
                                          Y[i * W + j] = v;
                                        });
}

// G[:, 0:ncols] = B' Y[:, 0:ncols] + [R_t | S_t | r_t | 0]
template <int MM, int E>
LQR_DEV void stage_hessian(const InstDesc& d, int t, const SweepLds& s, int ncols) {
  const int n = d.n, m = d.m, W = s.W;
  const LQR_GLOBAL double* Rt = gp(d.R + (size_t)t * m * m);
  const LQR_GLOBAL double* St = d.S ? gp(d.S + (size_t)t * m * n) : nullptr;
  const LQR_GLOBAL double* rt = gp(d.r + (size_t)t * m);
  double* G = s.G;
  const int mp = s.mp;
  pgemm_sub<E, true, false, false, false>(m, ncols, n, s.X, s.WX, s.Y, W, 0, s.X, s.WX, s.Y, W,
                                       [=](int i, int j, double v) {
                                         if (j < m) {
                                           v += Rt[i * m + j];
                                         } else if (j < m + n) {
                                           if (St) v += St[i * n + (j - m)];
                                         } else if (j == m + n) {
                                           v += rt[i];
                                         }
                                         G[j * mp + i] = v;
                                       });
}

// [P | p] <- [Q_t | q_t] + A'[PA | Pc+p] - Z'[Z | z], lower triangle computed
// and mirrored; optionally also written to the global outputs Pg, pg.
template <int MM, int E>
LQR_DEV void stage_value(const InstDesc& d, int t, const SweepLds& s, double* Pg, double* pg) {
  const int n = d.n, m = d.m, W = s.W;
  const LQR_GLOBAL double* Qt = gp(d.Q + (size_t)t * n * n);
  const LQR_GLOBAL double* qt = gp(d.q + (size_t)t * n);
  LQR_GLOBAL double* Pgg = gp(Pg);
  LQR_GLOBAL double* pgg = gp(pg);
  double* P = s.P;
  double* p = s.p;
  const int ldp = s.ldp;
  pgemm_sub<E, true, false, false, true>(n, n + 1, n, s.X + m, s.WX, s.Y + m, W, m, s.G + m * s.mp, s.mp, s.G + m * s.mp, s.mp,
      [=](int i, int j, double v) {
        if (j < n) {
          if (i >= j) {
            v += 0.5 * (Qt[i * n + j] + Qt[j * n + i]);
            P[i * ldp + j] = v;
            P[j * ldp + i] = v;
            if (Pgg) {
              Pgg[i * n + j] = v;
              Pgg[j * n + i] = v;
            }
          }
        } else {
          v += qt[i];
          p[i] = v;
          if (pgg) pgg[i] = v;
          if (!isfinite(v)) s.bad[1] = 1;  // non-finite value gradient
        }
      },
      SkipUpper{n});
}

// Plain Riccati recursion over stages [t0, t1) from the value (Pend, pend) at
// stage t1 (global memory). Per stage, with the Cholesky factor L of the input
// Hessian H_uu = R + B'PB and Z = L^{-1}[H_ux | h_u] (H_ux = S + B'PA,
// h_u = r + B'(Pc + p)):
//   [K | k] = -L^{-T} Z,   P <- Q + A'PA - Z_ux'Z_ux,   p <- q + A'(Pc+p) - Z_ux'z_h.
// Writes K_t, k_t and, when requested, chol_t, P_t, p_t for t in [t0, t1).
// Leaves the value at t0 in LDS (s.P, s.p). Returns a status code (see
// note_pivot; also LQR_INFO_NONFINITE for a non-finite value gradient),
// uniform across the workgroup.
template <int MM, int E>
LQR_DEV int plain_sweep(const InstDesc& d, int t0, int t1, const double* Pend, const double* pend,
                        const SweepLds& s) {
  const int n = d.n, m = d.m, WX = s.WX;
  if (threadIdx.x == 0) {
    s.bad[0] = 0;
    s.bad[1] = 0;
  }
  load_block(s.P, s.ldp, Pend, n, n, n);
  for (int i = threadIdx.x; i < n; i += kThreads) s.p[i] = pend[i];
  int fail = 0;
  double* dead = reinterpret_cast<double*>(s.bad) + 1;
  for (int t = t1 - 1; t >= t0; --t) {
    load_stage(d, t, s);
    __builtin_amdgcn_sched_barrier(0);  // keep the warming loads behind the staging waits
    const Touch next = touch_stage(d, t > t0 ? t - 1 : t);
    __syncthreads();
    stage_products<MM, E>(d, s);
    __syncthreads();
    stage_hessian<MM, E>(d, t, s, WX);
    __syncthreads();
    // L D L' of H_uu with the right-hand sides [H_ux | h_u | I]: Z = L^{-1}[H_ux | h_u]
    // into G, L^{-1} into G's first m columns (column q of L^{-1} in column q)
    ldl_columns<MM>(s.G, s.mp, m, n + 1, true, s.G, s.mp,
                    d.chol ? d.chol + (size_t)t * m * m : nullptr, s.E, s.bad);
    fail = note_pivot(fail, *s.bad, t);
    stage_value<MM, E>(d, t, s, d.P ? d.P + (size_t)t * n * n : nullptr,
                d.p ? d.p + (size_t)t * n : nullptr);
    {  // [K | k] = -H^{-1}[H_ux | h_u] = -(L^{-1})' Z
      LQR_GLOBAL double* Kt = gp(d.K + (size_t)t * m * n);
      LQR_GLOBAL double* kt = gp(d.k + (size_t)t * m);
      const int mp = s.mp;
      pgemm_sub<fp64_engine(E), false, false, false, true>(m, n + 1, 0, s.G, mp, s.G, mp, m, s.G, mp, s.G + m * mp, mp,
          [=](int i, int j, double v) {
            if (j < n)
              Kt[i * n + j] = v;
            else
              kt[i] = v;
          });
    }
    sink(next, dead);
    __syncthreads();
  }
  return (fail == 0 && s.bad[1]) ? LQR_INFO_NONFINITE : fail;
}

// Parametric (dual-form) sweep of a middle segment [t0, t1): the cost-to-go
// with zero terminal Hessian and a linear terminal price mu on x_{t1} is
//   V(x; mu) = 1/2 x'P0 x + (Gam mu + pbar)'x + psi'mu - 1/2 mu'Psi mu + const,
// and the segment's end state is dV/dmu = Gam'x + psi - Psi mu. P0, pbar follow
// the plain recursion from zero; per stage, with Z = L^{-1}[H_ux | h_u | B'Gam]
// (L the Cholesky factor of the input Hessian):
//   Psi += Z_W'Z_W,  psi += Gam'c - Z_W'z_h,  Gam <- A'Gam - Z_ux'Z_W
// (Gam' is the closed-loop transition of the segment). Writes
// P0 | Gam | Psi | pbar | psi to `out`. Returns as plain_sweep.
template <int MM, int E>
LQR_DEV int dual_sweep(const InstDesc& d, int t0, int t1, double* out, const SweepLds& s) {
  const int n = d.n, m = d.m, W = s.W, WX = s.WX;
  double* Gam = s.Y + WX;  // columns [WX, WX+n) of Y
  if (threadIdx.x == 0) *s.bad = 0;
  fill_block(s.P, s.ldp, n, n, 0.0, 0.0);
  fill_block(s.Psi, n, n, n, 0.0, 0.0);
  fill_block(Gam, W, n, n, 0.0, 1.0);
  for (int i = threadIdx.x; i < n; i += kThreads) {
    s.p[i] = 0.0;
    s.psi[i] = 0.0;
  }
  int fail = 0;
  double* dead = reinterpret_cast<double*>(s.bad) + 1;
  for (int t = t1 - 1; t >= t0; --t) {
    load_stage(d, t, s);
    __builtin_amdgcn_sched_barrier(0);  // keep the warming loads behind the staging waits
    const Touch next = touch_stage(d, t > t0 ? t - 1 : t);
    __syncthreads();
    stage_products<MM, E>(d, s);
    {  // gc = Gam' c_t (Gam of stage t+1)
      const double* X = s.X;
      for (int i = threadIdx.x; i < n; i += kThreads) s.gc[i] = col_dot(Gam, W, X + m + n, WX, i, n);
    }
    __syncthreads();
    stage_hessian<MM, E>(d, t, s, W);
    __syncthreads();
    ldl_columns<MM>(s.G, s.mp, m, 2 * n + 1, false, nullptr, 0, nullptr, s.E, s.bad);
    fail = note_pivot(fail, *s.bad, t);
    stage_value<MM, E>(d, t, s, nullptr, nullptr);
    {  // [psi-part | Psi-part] = Z_W' [z_h | Z_W]
      double* Psi = s.Psi;
      double* psi = s.psi;
      const double* gc = s.gc;
      const int mp = s.mp;
      pgemm_sub<E, false, true, false, false>(n, n + 1, m, s.G + WX * mp, mp, s.G + (m + n) * mp, mp, 0, s.G, mp, s.G, mp,
          [=](int i, int j, double v) {
            if (j == 0) {
              psi[i] += gc[i] - v;
            } else if (i >= j - 1) {
              const int jj = j - 1;
              const double nv = Psi[i * n + jj] + v;
              Psi[i * n + jj] = nv;
              Psi[jj * n + i] = nv;
            }
          },
          SkipUpperShift{n, 1});
    }
    __syncthreads();
    {  // Gam_new = A'Gam - Z_ux'Z_W  -> the (now free) P A region of Y
      double* Ynew = s.Y + m;
      const int mp = s.mp;
      pgemm_sub<E, true, false, false, true>(n, n, n, s.X + m, WX, Gam, W, m, s.G + m * mp, mp, s.G + WX * mp, mp,
          [=](int i, int j, double v) { Ynew[i * W + j] = v; });
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += kThreads) {
      const int i = e / n, j = e - i * n;
      Gam[i * W + j] = s.Y[i * W + m + j];
    }
    sink(next, dead);
  }
  __syncthreads();
  const int nn = n * n;
  store_block(out, n, s.P, s.ldp, n, n);
  store_block(out + nn, n, Gam, W, n, n);
  store_block(out + 2 * nn, n, s.Psi, n, n, n);
  for (int i = threadIdx.x; i < n; i += kThreads) {
    gp(out)[3 * nn + i] = s.p[i];
    gp(out)[3 * nn + n + i] = s.psi[i];
  }
  return fail;
}

// Streamed form of dual_sweep for segments whose resident layout exceeds
// the LDS: Gamma and Psi live in global memory (Psi accumulated in place in
// `out`, Gamma alternating between `out` and the scratch `gtmp`, n x n) and
// A_t is read from global memory by the products that use it. LDS holds P, p,
// [B_t | c_t], P[B_t | A_t | c_t] + [0 | 0 | p] and the Hessian block G.
// Same recursion and results as dual_sweep; LDS footprint sweep_lds_gs.
template <int MM, int E>
LQR_DEV int dual_sweep_gs(const InstDesc& d, int t0, int t1, double* out, double* gtmp,
                          double* smem) {
  const int n = d.n, m = d.m, nn = n * n;
  const int WX = m + 1, WY = m + n + 1, mp = MM + 1;
  const int ldp = p_ld(n);
  double* P = smem;              // n x n, leading dimension ldp
  double* p = P + n * ldp;
  double* X = p + n;             // n x (m+1): [B | c]
  double* Y = X + n * WX;        // n x (m+n+1): [PB | PA | Pc+p]
  double* G = Y + n * WY;        // mp x (m+2n+1) column-major
  double* Eb = G + mp * (m + 2 * n + 1);
  double* psi = Eb + 3 * MM;
  double* gc = psi + n;
  int* bad = reinterpret_cast<int*>(gc + n);
  double* Psi = out + 2 * nn;
  double* Gam = out + nn;
  double* Gn = gtmp;
  if (threadIdx.x == 0) *bad = 0;
  fill_block(P, ldp, n, n, 0.0, 0.0);
  for (int e = threadIdx.x; e < nn; e += kThreads) {  // Psi = 0, Gam = I (global)
    gp(Psi)[e] = 0.0;
    gp(Gam)[e] = (e / n == e % n) ? 1.0 : 0.0;
  }
  for (int i = threadIdx.x; i < n; i += kThreads) {
    p[i] = 0.0;
    psi[i] = 0.0;
  }
  int fail = 0;
  for (int t = t1 - 1; t >= t0; --t) {
    const double* At = d.A + (size_t)t * nn;
    const LQR_GLOBAL double* ct = gp(d.c + (size_t)t * n);
    const LQR_GLOBAL double* Rt = gp(d.R + (size_t)t * m * m);
    const LQR_GLOBAL double* St = d.S ? gp(d.S + (size_t)t * m * n) : nullptr;
    const LQR_GLOBAL double* rt = gp(d.r + (size_t)t * m);
    load_block(X, WX, d.B + (size_t)t * n * m, m, n, m);
    for (int i = threadIdx.x; i < n; i += kThreads) X[i * WX + m] = ct[i];
    __builtin_amdgcn_sched_barrier(0);  // keep the warming loads behind the staging waits
    const Touch next = touch_stage(d, t > t0 ? t - 1 : t);
    __syncthreads();
    // Y = P [B | A | c] + [0 | 0 | p]
    pgemm_sub<E, false, false, false, false>(n, m + 1, n, P, ldp, X, WX, 0, P, ldp, X, WX,
        [=](int i, int j, double v) {
          if (j < m) Y[i * WY + j] = v;
          else Y[i * WY + m + n] = v + p[i];
        });
    pgemm_sub<E, false, false, false, false>(n, n, n, P, ldp, At, n, 0, P, ldp, At, n,
        [=](int i, int j, double v) { Y[i * WY + m + j] = v; });
    // gc = Gam' c (Gam of stage t+1)
    for (int i = threadIdx.x; i < n; i += kThreads) gc[i] = col_dot(Gam, n, X + m, WX, i, n);
    __syncthreads();
    // G = B'[PB | PA | Pc+p | Gam] + [R | S | r | 0]
    pgemm_sub<E, true, false, false, false>(m, m + n + 1, n, X, WX, Y, WY, 0, X, WX, Y, WY,
        [=](int i, int j, double v) {
          if (j < m) v += Rt[i * m + j];
          else if (j < m + n) { if (St) v += St[i * n + (j - m)]; }
          else v += rt[i];
          G[j * mp + i] = v;
        });
    pgemm_sub<E, true, false, false, false>(m, n, n, X, WX, Gam, n, 0, X, WX, Gam, n,
        [=](int i, int j, double v) { G[(m + n + 1 + j) * mp + i] = v; });
    __syncthreads();
    ldl_columns<MM>(G, mp, m, 2 * n + 1, false, nullptr, 0, nullptr, Eb, bad);
    fail = note_pivot(fail, *bad, t);
    {  // [P | p] <- [Q | q] + A'[PA | Pc+p] - Z_ux'[Z_ux | z_h]
      const LQR_GLOBAL double* Qt = gp(d.Q + (size_t)t * nn);
      const LQR_GLOBAL double* qt = gp(d.q + (size_t)t * n);
      pgemm_sub<E, true, false, false, true>(n, n + 1, n, At, n, Y + m, WY, m, G + m * mp, mp,
          G + m * mp, mp,
          [=](int i, int j, double v) {
            if (j < n) {
              if (i >= j) {
                v += 0.5 * (Qt[i * n + j] + Qt[j * n + i]);
                P[i * ldp + j] = v;
                P[j * ldp + i] = v;
              }
            } else {
              p[i] = v + qt[i];
            }
          },
          SkipUpper{n});
    }
    {  // Psi += Z_W'Z_W (in place, global), psi += Gam'c - Z_W'z_h
      pgemm_sub<E, false, true, false, false>(n, n + 1, m, G + (m + n + 1) * mp, mp, G + (m + n) * mp, mp,
          0, G, mp, G, mp,
          [=, gPsi = gp(Psi)](int i, int j, double v) {
            if (j == 0) {
              psi[i] += gc[i] - v;
            } else if (i >= j - 1) {
              const int jj = j - 1;
              const double nv = gPsi[i * n + jj] + v;
              gPsi[i * n + jj] = nv;
              gPsi[jj * n + i] = nv;
            }
          },
          SkipUpperShift{n, 1});
    }
    // Gam <- A'Gam - Z_ux'Z_W into the other buffer
    pgemm_sub<E, true, false, false, true>(n, n, n, At, n, Gam, n, m, G + m * mp, mp,
        G + (m + n + 1) * mp, mp, [=, gGn = gp(Gn)](int i, int j, double v) { gGn[i * n + j] = v; });
    sink(next, reinterpret_cast<double*>(bad) + 1);
    __syncthreads();
    double* tmp = Gam;
    Gam = Gn;
    Gn = tmp;
  }
  __syncthreads();
  store_block(out, n, P, ldp, n, n);
  if (Gam != out + nn) store_block(out + nn, n, Gam, n, n, n);
  for (int i = threadIdx.x; i < n; i += kThreads) {
    gp(out)[3 * nn + i] = p[i];
    gp(out)[3 * nn + n + i] = psi[i];
  }
  __syncthreads();
  return fail;
}

// Rows `lane` of the column block [c0, c0 + cw) of an M (rows x cols, row
// stride ld) into registers r[0..15]; zero outside the matrix.
LQR_DEV void load_row_block(double (&r)[16], const double* M, int ld, int rows, int cols, int c0, int cw,
                            int lane) {
  const bool ok = lane < rows;
  const LQR_GLOBAL double* row = gp(M + (size_t)(ok ? lane : 0) * ld + c0);
#pragma unroll
  for (int q = 0; q < 16; ++q) r[q] = (ok && q < cw && c0 + q < cols) ? row[q] : 0.0;
}

// s + sum_q r[q] v_{c0+q} for q < cw, where v_c is held by lane c of the wave
// (c0 and cw wave-uniform, c0 + cw <= 64).
LQR_DEV double row_block_dot(const double (&r)[16], double v, int c0, int cw, double s) {
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q < cw) s = fma(r[q], readlane(v, c0 + q), s);
  return s;
}

// Forward simulation of stages [t0, t1) from x_{t0} = xs (global):
// u_t = K_t x_t + k_t, x_{t+1} = A_t x_t + B_t u_t + c_t (c_t = 0 when d.c is
// null); writes x_t, u_t
// (and lam_t = P_t x_t + p_t when requested), plus x_T (lam_T) if last.
// Returns LQR_INFO_NONFINITE (uniformly) if any value it wrote is not finite,
// else 0. n, m <= 64. Every wave holds the state in registers (lane i: x_i, u_i).
// Each matrix-vector product is split by columns over the waves (wave w takes
// a contiguous quarter of the columns, lane i row i); the partial sums meet in
// LDS and every wave adds them up in the same order, so a stage costs two
// barriers. The next stage's matrix rows are loaded into registers while the
// current stage is computed, which keeps global-memory latency off the chain.
// LDS: rollout_lds.
LQR_DEV int rollout(const InstDesc& d, int t0, int t1, const double* xs, bool last, double* smem) {
  const int n = d.n, m = d.m, T = d.T;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cn = (n + kWaves - 1) / kWaves, cm = (m + kWaves - 1) / kWaves;
  const int n0 = wave * cn, m0 = wave * cm;
  const bool rn = lane < n, rm = lane < m;
  const bool want_lam = d.lam != nullptr;
  double* part1 = smem;                 // [kWaves][128]: P x rows in [0, 64), K x rows in [64, 128)
  double* part2 = smem + kWaves * 128;  // [kWaves][64]: A x + B u
  double pP[16], pK[16], pA[16], pB[16];
  double bp = 0.0, bk = 0.0, bc = 0.0;  // p_t, k_t, c_t of row `lane`
#pragma unroll
  for (int q = 0; q < 16; ++q) pP[q] = pK[q] = pA[q] = pB[q] = 0.0;
  // value (P_t, p_t), gain (K_t, k_t) and dynamics (A_t, B_t, c_t) of stage t
  auto fetch_value = [&](int t) {
    load_row_block(pP, d.P + (size_t)t * n * n, n, n, n, n0, cn, lane);
    bp = rn ? gp(d.p)[(size_t)t * n + lane] : 0.0;
  };
  auto fetch_gain = [&](int t) {
    load_row_block(pK, d.K + (size_t)t * m * n, n, m, n, n0, cn, lane);
    bk = rm ? gp(d.k)[(size_t)t * m + lane] : 0.0;
  };
  auto fetch_dyn = [&](int t) {
    load_row_block(pA, d.A + (size_t)t * n * n, n, n, n, n0, cn, lane);
    load_row_block(pB, d.B + (size_t)t * n * m, m, n, m, m0, cm, lane);
    bc = (rn && d.c) ? gp(d.c)[(size_t)t * n + lane] : 0.0;
  };
  double x = rn ? gp(xs)[lane] : 0.0, u = 0.0;
  bool finite = true;  // every value this lane wrote so far
  if (t0 < t1) {
    if (want_lam) fetch_value(t0);
    fetch_gain(t0);
    fetch_dyn(t0);
  } else if (last && want_lam) {
    fetch_value(T);
  }
  for (int t = t0; t < t1; ++t) {
    const bool more = t + 1 < t1;
    if (wave == 0 && rn) gp(d.x)[(size_t)t * n + lane] = x;
    // partial P x and K x over this wave's columns
    part1[wave * 128 + lane] = want_lam ? row_block_dot(pP, x, n0, cn, 0.0) : 0.0;
    part1[wave * 128 + 64 + lane] = row_block_dot(pK, x, n0, cn, 0.0);
    const double cp = bp, ck = bk;
    if (want_lam && (more || last)) fetch_value(t + 1);
    if (more) fetch_gain(t + 1);
    __syncthreads();
    double sl = 0.0, su = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      sl += part1[w * 128 + lane];
      su += part1[w * 128 + 64 + lane];
    }
    if (want_lam && wave == 2 && rn) {
      gp(d.lam)[(size_t)t * n + lane] = cp + sl;
      finite = finite && isfinite(cp + sl);
    }
    u = rm ? ck + su : 0.0;
    finite = finite && isfinite(x) && isfinite(u);
    if (wave == 1 && rm) gp(d.u)[(size_t)t * m + lane] = u;
    // partial A x + B u
    part2[wave * 64 + lane] = row_block_dot(pB, u, m0, cm, row_block_dot(pA, x, n0, cn, 0.0));
    const double cb = bc;
    if (more) fetch_dyn(t + 1);
    __syncthreads();
    double sx = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) sx += part2[w * 64 + lane];
    x = rn ? cb + sx : 0.0;
  }
  if (last) {
    if (wave == 0 && rn) gp(d.x)[(size_t)T * n + lane] = x;
    finite = finite && isfinite(x);
    if (want_lam) {
      part1[wave * 128 + lane] = row_block_dot(pP, x, n0, cn, 0.0);
      __syncthreads();
      double sl = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) sl += part1[w * 128 + lane];
      if (wave == 2 && rn) {
        gp(d.lam)[(size_t)T * n + lane] = bp + sl;
        finite = finite && isfinite(bp + sl);
      }
    }
  }
  // any lane of any wave: one ballot per wave, met in LDS after the partial sums
  // (no static LDS: every byte of the workgroup's LDS may be dynamic)
  int* anybad = reinterpret_cast<int*>(smem + kWaves * 192);
  const bool wbad = __ballot(!finite) != 0ull;
  if (lane == 0) anybad[wave] = wbad ? 1 : 0;
  __syncthreads();
  int bad = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) bad |= anybad[w];
  __syncthreads();
  return bad ? LQR_INFO_NONFINITE : 0;
}

// Terminal value P_T = Q_T, p_T = q_T into the outputs (if requested).
LQR_DEV void write_terminal(const InstDesc& d) {
  const int n = d.n, T = d.T;
  if (d.P) store_block(d.P + (size_t)T * n * n, n, d.Q + (size_t)T * n * n, n, n, n);
  if (d.p)
    for (int i = threadIdx.x; i < n; i += kThreads) gp(d.p)[(size_t)T * n + i] = gp(d.q)[(size_t)T * n + i];
}

template <int MM, int E>
LQR_DEV void phase1_item(const InstDesc& d, int seg, double* smem) {
  const int n = d.n, m = d.m, T = d.T, J = d.J;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  int fail;
  if (seg < J - 1) {
    if (sweep_lds(n, m, true, MM) <= kLdsSweepMax) {
      SweepLds s = carve_sweep(smem, n, m, true, MM);
      fail = dual_sweep<MM, E>(d, t0, t1, ws_seg(d.ws, n, seg), s);
    } else {
      double* gtmp = ws_scan(d.ws, n, J, 0) + (size_t)seg * seg_stride(n);
      fail = dual_sweep_gs<MM, E>(d, t0, t1, ws_seg(d.ws, n, seg), gtmp, smem);
    }
  } else {
    SweepLds s = carve_sweep(smem, n, m, false, MM);
    write_terminal(d);
    fail = plain_sweep<MM, E>(d, t0, t1, d.Q + (size_t)T * n * n, d.q + (size_t)T * n, s);
    double* b = ws_bnd(d.ws, n, J, J - 1);
    store_block(b, n, s.P, s.ldp, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) b[n * n + i] = s.p[i];
  }
  if (threadIdx.x == 0) {
    d.fail[seg] = fail;
    if (seg == 0) d.fail[J] = 0;  // the linking-failure word, raised by phase 2
  }
}

// Linking solve. With (Pn, pn) the exact value at t_{j+1} and N = I + Psi_j Pn:
//   [F | f] = N^{-1} [Gam_j' | psi_j - Psi_j pn]   (explicit inverse, wg_invert)
//   P_{t_j} = P0_j + Gam_j Pn F,   p_{t_j} = pbar_j + Gam_j (pn + Pn f)
// which is the elimination of x_{t_{j+1}} and the link multiplier
// mu_j = (I + Pn Psi_j)^{-1}(Pn (Gam_j' x + psi_j) + pn) from the segment's
// value; forward, x_{t_{j+1}} = F x_{t_j} + f. Blocks in LDS are
// n x ld_odd(n), row-major unless noted.
template <int MN, int E>
LQR_DEV void couple_item(const InstDesc& d, double* smem) {
  const int n = d.n, J = d.J;
  const int L = ld_odd(n), blk = n * L;
  double* sPn = smem;        // exact value at t_{j+1}
  double* sA1 = sPn + blk;   // Psi, then Gam
  double* sN = sA1 + blk;    // N, column-major -> its inverse in place -> T1 = Pn F
  double* sF = sN + blk;     // F' (row c holds column c of F)
  double* spn = sF + blk;
  double* sv = spn + n;      // w = psi - Psi pn, then pn + Pn f
  double* sf = sv + n;
  double* sx = sf + n;
  double* sxn = sx + n;
  const InvExchange ix = carve_inv_exchange(sxn + n);
  int* flag = reinterpret_cast<int*>(sxn + n + kInvExchangeDoubles);

  if (threadIdx.x == 0) {
    int f = 0;
    for (int j = 0; j < J; ++j) f = combine_info(f, d.fail[j]);
    flag[0] = f;  // stage failure (or non-finite value) from phase 1
    flag[1] = 0;  // linking failure
  }
  {
    const double* bl = ws_bnd(d.ws, n, J, J - 1);
    load_block(sPn, L, bl, n, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) spn[i] = gp(bl)[n * n + i];
  }
  for (int j = J - 2; j >= 0; --j) {
    const double* sg = ws_seg(d.ws, n, j);
    const LQR_GLOBAL double* P0 = gp(sg);
    const double* Gam = sg + n * n;
    const double* Psi = sg + 2 * n * n;
    const LQR_GLOBAL double* pbar = gp(sg + 3 * n * n);
    const LQR_GLOBAL double* psi = pbar + n;
    load_block(sA1, L, Psi, n, n, n);
    __syncthreads();
    pgemm_sub<fp64_engine(E), false, false, false, false>(n, n, n, sA1, L, sPn, L, 0, sA1, L, sPn, L,
                                          [=](int i, int jj, double v) {
                                            sN[jj * L + i] = v + (i == jj ? 1.0 : 0.0);
                                          });
    gemv_wave(1, n, n, sA1, L, spn, [=](int i, double v) { sv[i] = psi[i] - v; });
    __syncthreads();
    load_block(sA1, L, Gam, n, n, n);  // Psi no longer needed
    const int bad = wg_invert<MN>(sN, L, n, sN, L, ix);
    if (threadIdx.x == 0 && bad && !flag[1]) flag[1] = LQR_INFO_COUPLING + j;
    // [F | f] = N^{-1} [Gam' | w], kept in LDS and written to the workspace
    // (F column-major) for the forward pass: F' = Gam N^{-T}
    LQR_GLOBAL double* lk = gp(ws_link(d.ws, n, J, j));
    pgemm_sub<fp64_engine(E), false, false, false, false>(n, n, n, sA1, L, sN, L, 0, sA1, L, sN, L,
        [=](int c, int i, double v) {
          sF[c * L + i] = v;
          lk[c * n + i] = v;
        });
    gemv_cm_wave(1, n, n, sN, L, sv, [=](int i, double v) {
      sf[i] = v;
      lk[n * n + i] = v;
    });
    __syncthreads();
    // T1 = Pn F -> sN ;  v = pn + Pn f
    pgemm_sub<fp64_engine(E), false, true, false, false>(n, n, n, sPn, L, sF, L, 0, sPn, L, sF, L,
                                         [=](int i, int jj, double v) { sN[i * L + jj] = v; });
    gemv_wave(1, n, n, sPn, L, sf, [=](int i, double v) { sv[i] = spn[i] + v; });
    __syncthreads();
    pgemm_sub<fp64_engine(E), false, false, false, false>(n, n, n, sA1, L, sN, L, 0, sA1, L, sN, L,
        [=](int i, int jj, double v) {
          if (i >= jj) {
            v += 0.5 * (P0[i * n + jj] + P0[jj * n + i]);
            sPn[i * L + jj] = v;
            sPn[jj * L + i] = v;
          }
        },
        SkipUpper{n});
    gemv_wave(1, n, n, sA1, L, sv, [=](int i, double v) { spn[i] = pbar[i] + v; });
    __syncthreads();
    double* b = ws_bnd(d.ws, n, J, j);
    store_block(b, n, sPn, L, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) gp(b)[n * n + i] = spn[i];
  }
  // forward over the boundaries: x_{t_0} = x0, x_{t_{j+1}} = F_j x_{t_j} + f_j
  for (int i = threadIdx.x; i < n; i += kThreads) {
    sx[i] = gp(d.x0)[i];
    gp(ws_bnd(d.ws, n, J, 0))[n * n + n + i] = gp(d.x0)[i];
  }
  __syncthreads();
  for (int j = 0; j < J - 1; ++j) {
    const double* lk = ws_link(d.ws, n, J, j);
    const LQR_GLOBAL double* lkf = gp(lk + n * n);
    gemv_cm_wave(0, n, n, lk, n, sx, [=](int i, double v) { sxn[i] = lkf[i] + v; });
    __syncthreads();
    LQR_GLOBAL double* xb = gp(ws_bnd(d.ws, n, J, j + 1) + n * n + n);
    for (int i = threadIdx.x; i < n; i += kThreads) {
      sx[i] = sxn[i];
      xb[i] = sxn[i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *d.info = flag[0] ? flag[0] : flag[1];
}

template <int MM, int E>
LQR_DEV void phase3_item(const InstDesc& d, int seg, double* smem) {
  const int n = d.n, m = d.m, T = d.T, J = d.J;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  if (seg < J - 1) {
    SweepLds s = carve_sweep(smem, n, m, false, MM);
    const double* b = ws_bnd(d.ws, n, J, seg + 1);
    const int fail = plain_sweep<MM, E>(d, t0, t1, b, b + n * n, s);
    if (fail && threadIdx.x == 0) report_info(d.info, fail);
  }
  const int nf = rollout(d, t0, t1, ws_bnd(d.ws, n, J, seg) + n * n + n, seg == J - 1, smem);
  if (nf && threadIdx.x == 0) report_info(d.info, nf);
}

template <int MM, int E>
LQR_DEV void serial_item(const InstDesc& d, double* smem) {
  const int n = d.n, m = d.m, T = d.T;
  SweepLds s = carve_sweep(smem, n, m, false, MM);
  write_terminal(d);
  const int fail = plain_sweep<MM, E>(d, 0, T, d.Q + (size_t)T * n * n, d.q + (size_t)T * n, s);
  const int nf = rollout(d, 0, T, d.x0, true, smem);
  if (threadIdx.x == 0) *d.info = combine_info(fail, nf);
}


// Descriptor of the work a workgroup runs: a single instance passed by value,
// or an (instance, segment) item of a batched launch's device tables.
LQR_DEV void select_item(const InstDesc& single, const InstDesc* descs, const WorkItem* items,
                         InstDesc& d, int& seg) {
  if (items) {
    const WorkItem w = items[blockIdx.x];
    d = descs[w.inst];
    seg = w.seg;
  } else if (descs) {
    d = descs[blockIdx.x];
    seg = 0;
  } else {
    d = single;
    seg = blockIdx.x;
  }
}

}  // namespace lqr
