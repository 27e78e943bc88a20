// Kernels of the parallel Riccati recursion (FP64), gfx950.
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
#include <hip/hip_runtime.h>

#include "lqr_kernels.h"
#include "lqr_layout.h"
#include "wg_linalg.h"

namespace lqr {

namespace {

struct SweepLds {
  double *P, *p, *X, *Y, *G, *d, *Psi, *psi, *gc;
  int* bad;
  int WX, W;
};

LQR_DEV SweepLds carve_sweep(double* smem, int n, int m, bool dual) {
  SweepLds s;
  s.WX = m + n + 1;
  s.W = sweep_w(n, m, dual);
  double* q = smem;
  s.P = q; q += n * n;
  s.p = q; q += n;
  s.X = q; q += n * s.WX;
  s.Y = q; q += n * s.W;
  s.G = q; q += m * s.W;
  s.d = q; q += m;
  s.Psi = s.psi = s.gc = nullptr;
  if (dual) {
    s.Psi = q; q += n * n;
    s.psi = q; q += n;
    s.gc = q; q += n;
  }
  s.bad = reinterpret_cast<int*>(q);
  return s;
}

// Stage inputs into LDS: X = [B_t | A_t | c_t].
LQR_DEV void load_stage(const InstDesc& d, int t, const SweepLds& s) {
  const int n = d.n, m = d.m;
  load_block(s.X, s.WX, d.B + (size_t)t * n * m, m, n, m);
  load_block(s.X + m, s.WX, d.A + (size_t)t * n * n, n, n, n);
  const double* ct = d.c + (size_t)t * n;
  for (int i = threadIdx.x; i < n; i += kThreads) s.X[i * s.WX + m + n] = ct[i];
}

// Y[:, 0:WX] = P [B | A | c] + [0 | 0 | p]
LQR_DEV void stage_products(const InstDesc& d, const SweepLds& s) {
  const int n = d.n, m = d.m, WX = s.WX, W = s.W;
  double* Y = s.Y;
  const double* p = s.p;
  gemm<4, 4, false, false>(n, WX, n, s.P, n, s.X, WX, [=](int i, int j, double v) {
    if (j == m + n) v += p[i];
    Y[i * W + j] = v;
  });
}

// G[:, 0:ncols] = B' Y[:, 0:ncols] + [R_t | S_t | r_t | 0]
LQR_DEV void stage_hessian(const InstDesc& d, int t, const SweepLds& s, int ncols) {
  const int n = d.n, m = d.m, W = s.W;
  const double* Rt = d.R + (size_t)t * m * m;
  const double* St = d.S ? d.S + (size_t)t * m * n : nullptr;
  const double* rt = d.r + (size_t)t * m;
  double* G = s.G;
  gemm<4, 4, true, false>(m, ncols, n, s.X, s.WX, s.Y, W, [=](int i, int j, double v) {
    if (j < m) {
      v += Rt[i * m + j];
    } else if (j < m + n) {
      if (St) v += St[i * n + (j - m)];
    } else if (j == m + n) {
      v += rt[i];
    }
    G[i * W + j] = v;
  });
}

// [P | p] <- [Q_t | q_t] + A'[PA | Pc+p] - Z'[Z | z], lower triangle computed
// and mirrored; optionally also written to the global outputs Pg, pg.
LQR_DEV void stage_value(const InstDesc& d, int t, const SweepLds& s, double* Pg, double* pg) {
  const int n = d.n, m = d.m, W = s.W;
  const double* Qt = d.Q + (size_t)t * n * n;
  const double* qt = d.q + (size_t)t * n;
  double* P = s.P;
  double* p = s.p;
  gemm_sub<4, 4, true, false, true, false>(
      n, n + 1, n, s.X + m, s.WX, s.Y + m, W, m, s.G + m, W, s.G + m, W,
      [=](int i, int j, double v) {
        if (j < n) {
          if (i >= j) {
            v += 0.5 * (Qt[i * n + j] + Qt[j * n + i]);
            P[i * n + j] = v;
            P[j * n + i] = v;
            if (Pg) {
              Pg[i * n + j] = v;
              Pg[j * n + i] = v;
            }
          }
        } else {
          v += qt[i];
          p[i] = v;
          if (pg) pg[i] = v;
        }
      },
      SkipUpper<4, 4>{n});
}

// Plain Riccati recursion over stages [t0, t1) from the value (Pend, pend) at
// stage t1 (global memory). Writes K_t, k_t and, when requested, chol_t, P_t,
// p_t for t in [t0, t1). Leaves the value at t0 in LDS (s.P, s.p). Returns
// (largest failing stage) + 1, or 0; uniform across the workgroup.
LQR_DEV int plain_sweep(const InstDesc& d, int t0, int t1, const double* Pend, const double* pend,
                        const SweepLds& s) {
  const int n = d.n, m = d.m, W = s.W, WX = s.WX;
  if (threadIdx.x == 0) *s.bad = 0;
  load_block(s.P, n, Pend, n, n, n);
  for (int i = threadIdx.x; i < n; i += kThreads) s.p[i] = pend[i];
  int fail = 0;
  for (int t = t1 - 1; t >= t0; --t) {
    load_stage(d, t, s);
    __syncthreads();
    stage_products(d, s);
    __syncthreads();
    stage_hessian(d, t, s, WX);
    __syncthreads();
    ldl_forward(s.G, W, m, WX, 0, s.d, s.bad);
    if (!fail && *s.bad) fail = t + 1;
    ldl_scale(s.G, W, m, WX, 0, s.d);
    __syncthreads();
    stage_value(d, t, s, d.P ? d.P + (size_t)t * n * n : nullptr,
                d.p ? d.p + (size_t)t * n : nullptr);
    __syncthreads();
    // [K | k] = -H^{-1}[S + B'PA | r + B'(Pc+p)]: back substitution with L'
    ltrsv_cols(s.G, W, m, 0, m, m + n + 1);
    __syncthreads();
    double* Kt = d.K + (size_t)t * m * n;
    double* kt = d.k + (size_t)t * m;
    for (int e = threadIdx.x; e < m * n; e += kThreads) {
      const int i = e / n, j = e - i * n;
      Kt[e] = -s.G[i * W + m + j];
    }
    for (int i = threadIdx.x; i < m; i += kThreads) kt[i] = -s.G[i * W + m + n];
    if (d.chol) {
      double* Lt = d.chol + (size_t)t * m * m;
      for (int e = threadIdx.x; e < m * m; e += kThreads) {
        const int i = e / m, j = e - i * m;
        Lt[e] = (i >= j) ? s.G[j * W + i] : 0.0;
      }
    }
  }
  __syncthreads();
  return fail;
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
LQR_DEV int dual_sweep(const InstDesc& d, int t0, int t1, double* out, const SweepLds& s) {
  const int n = d.n, m = d.m, W = s.W, WX = s.WX;
  double* Gam = s.Y + WX;  // columns [WX, WX+n) of Y
  if (threadIdx.x == 0) *s.bad = 0;
  fill_block(s.P, n, n, n, 0.0, 0.0);
  fill_block(s.Psi, n, n, n, 0.0, 0.0);
  fill_block(Gam, W, n, n, 0.0, 1.0);
  for (int i = threadIdx.x; i < n; i += kThreads) {
    s.p[i] = 0.0;
    s.psi[i] = 0.0;
  }
  int fail = 0;
  for (int t = t1 - 1; t >= t0; --t) {
    load_stage(d, t, s);
    __syncthreads();
    stage_products(d, s);
    {  // gc = Gam' c_t (Gam of stage t+1)
      const double* X = s.X;
      for (int i = threadIdx.x; i < n; i += kThreads) {
        double a = 0.0;
        for (int k = 0; k < n; ++k) a = fma(Gam[k * W + i], X[k * WX + m + n], a);
        s.gc[i] = a;
      }
    }
    __syncthreads();
    stage_hessian(d, t, s, W);
    __syncthreads();
    ldl_forward(s.G, W, m, W, 0, s.d, s.bad);
    if (!fail && *s.bad) fail = t + 1;
    ldl_scale(s.G, W, m, W, 0, s.d);
    __syncthreads();
    stage_value(d, t, s, nullptr, nullptr);
    {  // [psi-part | Psi-part] = Z_W' [z_h | Z_W]
      double* Psi = s.Psi;
      double* psi = s.psi;
      const double* gc = s.gc;
      gemm<4, 4, true, false>(
          n, n + 1, m, s.G + WX, W, s.G + m + n, W,
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
          SkipUpperShift<4, 4>{n, 1});
    }
    __syncthreads();
    {  // Gam_new = A'Gam - Z_ux'Z_W  -> the (now free) P A region of Y
      double* Ynew = s.Y + m;
      gemm_sub<4, 4, true, false, true, false>(
          n, n, n, s.X + m, WX, Gam, W, m, s.G + m, W, s.G + WX, W,
          [=](int i, int j, double v) { Ynew[i * W + j] = v; });
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += kThreads) {
      const int i = e / n, j = e - i * n;
      Gam[i * W + j] = s.Y[i * W + m + j];
    }
  }
  __syncthreads();
  const int nn = n * n;
  store_block(out, n, s.P, n, n, n);
  store_block(out + nn, n, Gam, W, n, n);
  store_block(out + 2 * nn, n, s.Psi, n, n, n);
  for (int i = threadIdx.x; i < n; i += kThreads) {
    out[3 * nn + i] = s.p[i];
    out[3 * nn + n + i] = s.psi[i];
  }
  return fail;
}

// Forward simulation of stages [t0, t1) from x_{t0} = xs (global):
// u_t = K_t x_t + k_t, x_{t+1} = A_t x_t + B_t u_t + c_t; writes x_t, u_t
// (and lam_t = P_t x_t + p_t when requested), plus x_T (lam_T) if last.
LQR_DEV void rollout(const InstDesc& d, int t0, int t1, const double* xs, bool last, double* smem) {
  const int n = d.n, m = d.m;
  double* sx = smem;
  double* sxn = smem + n;
  double* su = smem + 2 * n;
  for (int i = threadIdx.x; i < n; i += kThreads) sx[i] = xs[i];
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    double* xt = d.x + (size_t)t * n;
    for (int i = threadIdx.x; i < n; i += kThreads) xt[i] = sx[i];
    if (d.lam) {
      const double* pt = d.p + (size_t)t * n;
      double* lt = d.lam + (size_t)t * n;
      gemv2(n, n, d.P + (size_t)t * n * n, n, sx, 0, sx, 0, sx,
            [=](int i, double v) { lt[i] = pt[i] + v; });
    }
    const double* kt = d.k + (size_t)t * m;
    double* ut = d.u + (size_t)t * m;
    gemv2(m, n, d.K + (size_t)t * m * n, n, sx, 0, sx, 0, sx, [=](int i, double v) {
      v += kt[i];
      su[i] = v;
      ut[i] = v;
    });
    __syncthreads();
    const double* ct = d.c + (size_t)t * n;
    gemv2(n, n, d.A + (size_t)t * n * n, n, sx, m, d.B + (size_t)t * n * m, m, su,
          [=](int i, double v) { sxn[i] = ct[i] + v; });
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kThreads) sx[i] = sxn[i];
    __syncthreads();
  }
  if (last) {
    double* xT = d.x + (size_t)d.T * n;
    for (int i = threadIdx.x; i < n; i += kThreads) xT[i] = sx[i];
    if (d.lam) {
      const double* pT = d.p + (size_t)d.T * n;
      double* lT = d.lam + (size_t)d.T * n;
      gemv2(n, n, d.P + (size_t)d.T * n * n, n, sx, 0, sx, 0, sx,
            [=](int i, double v) { lT[i] = pT[i] + v; });
    }
  }
}

// Terminal value P_T = Q_T, p_T = q_T into the outputs (if requested).
LQR_DEV void write_terminal(const InstDesc& d) {
  const int n = d.n, T = d.T;
  if (d.P) store_block(d.P + (size_t)T * n * n, n, d.Q + (size_t)T * n * n, n, n, n);
  if (d.p)
    for (int i = threadIdx.x; i < n; i += kThreads) d.p[(size_t)T * n + i] = d.q[(size_t)T * n + i];
}

LQR_DEV void phase1_item(const InstDesc& d, int seg, double* smem) {
  const int n = d.n, m = d.m, T = d.T, J = d.J;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  int fail;
  if (seg < J - 1) {
    SweepLds s = carve_sweep(smem, n, m, true);
    fail = dual_sweep(d, t0, t1, ws_seg(d.ws, n, seg), s);
  } else {
    SweepLds s = carve_sweep(smem, n, m, false);
    write_terminal(d);
    fail = plain_sweep(d, t0, t1, d.Q + (size_t)T * n * n, d.q + (size_t)T * n, s);
    double* b = ws_bnd(d.ws, n, J, J - 1);
    store_block(b, n, s.P, n, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) b[n * n + i] = s.p[i];
  }
  if (threadIdx.x == 0) d.fail[seg] = fail;
}

// Linking solve. With (Pn, pn) the exact value at t_{j+1} and N = I + Psi_j Pn:
//   [F | f] = N^{-1} [Gam_j' | psi_j - Psi_j pn]       (Gauss-Jordan, row pivoting)
//   P_{t_j} = P0_j + Gam_j Pn F,   p_{t_j} = pbar_j + Gam_j (pn + Pn f)
// which is the elimination of x_{t_{j+1}} and the link multiplier
// mu_j = (I + Pn Psi_j)^{-1}(Pn (Gam_j' x + psi_j) + pn) from the segment's
// value; forward, x_{t_{j+1}} = F x_{t_j} + f.
LQR_DEV void couple_item(const InstDesc& d, double* smem) {
  const int n = d.n, J = d.J, LDN = 2 * n + 1;
  double* sPn = smem;
  double* spn = sPn + n * n;
  double* sA1 = spn + n;
  double* sN = sA1 + n * n;
  double* sv = sN + n * LDN;
  double* sf = sv + n;
  double* sx = sf + n;
  double* sxn = sx + n;
  double* sdp = sxn + n;
  int* ipiv = reinterpret_cast<int*>(sdp + n);
  int* used = ipiv + n;
  int* flag = used + n;

  if (threadIdx.x == 0) {
    int f = 0;
    for (int j = 0; j < J; ++j) f = max(f, d.fail[j]);
    flag[0] = f;  // stage failure from phase 1
    flag[1] = 0;  // linking failure
  }
  {
    const double* bl = ws_bnd(d.ws, n, J, J - 1);
    load_block(sPn, n, bl, n, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) spn[i] = bl[n * n + i];
  }
  for (int j = J - 2; j >= 0; --j) {
    const double* sg = ws_seg(d.ws, n, j);
    const double* P0 = sg;
    const double* Gam = sg + n * n;
    const double* Psi = sg + 2 * n * n;
    const double* pbar = sg + 3 * n * n;
    const double* psi = pbar + n;
    load_block(sA1, n, Psi, n, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) used[i] = 0;
    __syncthreads();
    gemm<4, 4, false, false>(n, n, n, sA1, n, sPn, n, [=](int i, int jj, double v) {
      sN[i * LDN + jj] = v + (i == jj ? 1.0 : 0.0);
    });
    load_block_t(sN + n, LDN, Gam, n, n, n);
    gemv2(n, n, sA1, n, spn, 0, spn, 0, spn, [=](int i, double v) { sN[i * LDN + 2 * n] = psi[i] - v; });
    __syncthreads();
    load_block(sA1, n, Gam, n, n, n);
    for (int k = 0; k < n; ++k) {
      if (threadIdx.x < 64) {
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int i = threadIdx.x; i < n; i += 64) {
          if (used[i]) continue;
          double a = fabs(sN[i * LDN + k]);
          if (!(a <= 1.7976931348623157e308)) a = __builtin_inf();
          if (a > best || (a == best && i < bi)) {
            best = a;
            bi = i;
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (threadIdx.x == 0) {
          double dk = sN[bi * LDN + k];
          if (!(dk != 0.0) || !isfinite(dk)) {
            if (!flag[1]) flag[1] = LQR_INFO_COUPLING + j;
            dk = qnan<double>();
          }
          ipiv[k] = bi;
          sdp[k] = dk;
          used[bi] = 1;
        }
      }
      __syncthreads();
      const int pr = ipiv[k];
      const double inv = 1.0 / sdp[k];
      const int nc = LDN - k - 1;  // columns k+1 .. 2n
      for (int e = threadIdx.x; e < n * nc; e += kThreads) {
        const int i = e / nc, jc = k + 1 + (e - i * nc);
        if (i == pr) continue;
        sN[i * LDN + jc] = fma(-sN[i * LDN + k] * inv, sN[pr * LDN + jc], sN[i * LDN + jc]);
      }
      __syncthreads();
    }
    {  // unpermute and scale: F -> sN[:, 0:n], f -> sf; also to the workspace
      double* lk = ws_link(d.ws, n, J, j);
      for (int e = threadIdx.x; e < n * (n + 1); e += kThreads) {
        const int k = e / (n + 1), c = e - k * (n + 1);
        const double v = sN[ipiv[k] * LDN + n + c] / sdp[k];
        if (c < n) {
          sN[k * LDN + c] = v;
          lk[k * n + c] = v;
        } else {
          sf[k] = v;
          lk[n * n + k] = v;
        }
      }
    }
    __syncthreads();
    gemm<4, 4, false, false>(n, n, n, sPn, n, sN, LDN, [=](int i, int jj, double v) {
      sN[i * LDN + n + jj] = v;
    });
    gemv2(n, n, sPn, n, sf, 0, sf, 0, sf, [=](int i, double v) { sv[i] = spn[i] + v; });
    __syncthreads();
    gemm<4, 4, false, false>(
        n, n, n, sA1, n, sN + n, LDN,
        [=](int i, int jj, double v) {
          if (i >= jj) {
            v += 0.5 * (P0[i * n + jj] + P0[jj * n + i]);
            sPn[i * n + jj] = v;
            sPn[jj * n + i] = v;
          }
        },
        SkipUpper<4, 4>{n});
    gemv2(n, n, sA1, n, sv, 0, sv, 0, sv, [=](int i, double v) { spn[i] = pbar[i] + v; });
    __syncthreads();
    double* b = ws_bnd(d.ws, n, J, j);
    store_block(b, n, sPn, n, n, n);
    for (int i = threadIdx.x; i < n; i += kThreads) b[n * n + i] = spn[i];
  }
  // forward over the boundaries: x_{t_0} = x0, x_{t_{j+1}} = F_j x_{t_j} + f_j
  for (int i = threadIdx.x; i < n; i += kThreads) {
    sx[i] = d.x0[i];
    ws_bnd(d.ws, n, J, 0)[n * n + n + i] = d.x0[i];
  }
  __syncthreads();
  for (int j = 0; j < J - 1; ++j) {
    const double* lk = ws_link(d.ws, n, J, j);
    gemv2(n, n, lk, n, sx, 0, sx, 0, sx, [=](int i, double v) { sxn[i] = lk[n * n + i] + v; });
    __syncthreads();
    double* xb = ws_bnd(d.ws, n, J, j + 1) + n * n + n;
    for (int i = threadIdx.x; i < n; i += kThreads) {
      sx[i] = sxn[i];
      xb[i] = sxn[i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *d.info = flag[0] ? flag[0] : flag[1];
}

LQR_DEV void phase3_item(const InstDesc& d, int seg, double* smem) {
  const int n = d.n, m = d.m, T = d.T, J = d.J;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  if (seg < J - 1) {
    SweepLds s = carve_sweep(smem, n, m, false);
    const double* b = ws_bnd(d.ws, n, J, seg + 1);
    const int fail = plain_sweep(d, t0, t1, b, b + n * n, s);
    if (fail && threadIdx.x == 0) atomicMax(d.info, fail);
  }
  rollout(d, t0, t1, ws_bnd(d.ws, n, J, seg) + n * n + n, seg == J - 1, smem);
}

LQR_DEV void serial_item(const InstDesc& d, double* smem) {
  const int n = d.n, m = d.m, T = d.T;
  SweepLds s = carve_sweep(smem, n, m, false);
  write_terminal(d);
  const int fail = plain_sweep(d, 0, T, d.Q + (size_t)T * n * n, d.q + (size_t)T * n, s);
  rollout(d, 0, T, d.x0, true, smem);
  if (threadIdx.x == 0) *d.info = fail;
}

}  // namespace

__global__ __launch_bounds__(kThreads) void k_phase1(InstDesc d) {
  extern __shared__ double smem[];
  phase1_item(d, blockIdx.x, smem);
}
__global__ __launch_bounds__(kThreads) void k_phase2(InstDesc d) {
  extern __shared__ double smem[];
  couple_item(d, smem);
}
__global__ __launch_bounds__(kThreads) void k_phase3(InstDesc d) {
  extern __shared__ double smem[];
  phase3_item(d, blockIdx.x, smem);
}
__global__ __launch_bounds__(kThreads) void k_serial(InstDesc d) {
  extern __shared__ double smem[];
  serial_item(d, smem);
}

__global__ __launch_bounds__(kThreads) void k_phase1_b(const InstDesc* descs, const WorkItem* items) {
  extern __shared__ double smem[];
  const WorkItem w = items[blockIdx.x];
  phase1_item(descs[w.inst], w.seg, smem);
}
__global__ __launch_bounds__(kThreads) void k_phase2_b(const InstDesc* descs) {
  extern __shared__ double smem[];
  couple_item(descs[blockIdx.x], smem);
}
__global__ __launch_bounds__(kThreads) void k_phase3_b(const InstDesc* descs, const WorkItem* items) {
  extern __shared__ double smem[];
  const WorkItem w = items[blockIdx.x];
  phase3_item(descs[w.inst], w.seg, smem);
}
__global__ __launch_bounds__(kThreads) void k_serial_b(const InstDesc* descs) {
  extern __shared__ double smem[];
  serial_item(descs[blockIdx.x], smem);
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
static hipError_t allow_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_parallel(const InstDesc& d, size_t lds1, size_t lds2, size_t lds3,
                           hipStream_t stream) {
  hipError_t e;
  if ((e = allow_lds((const void*)k_phase1, lds1)) != hipSuccess) return e;
  if ((e = allow_lds((const void*)k_phase2, lds2)) != hipSuccess) return e;
  if ((e = allow_lds((const void*)k_phase3, lds3)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_phase1, dim3(d.J), dim3(kThreads), lds1, stream, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_phase2, dim3(1), dim3(kThreads), lds2, stream, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_phase3, dim3(d.J), dim3(kThreads), lds3, stream, d);
  return hipGetLastError();
}

hipError_t launch_serial(const InstDesc& d, size_t lds, hipStream_t stream) {
  hipError_t e;
  if ((e = allow_lds((const void*)k_serial, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_serial, dim3(1), dim3(kThreads), lds, stream, d);
  return hipGetLastError();
}

hipError_t launch_parallel_batched(const InstDesc* descs, const WorkItem* items, int nitems,
                                   int ninst, size_t lds1, size_t lds2, size_t lds3,
                                   hipStream_t stream) {
  hipError_t e;
  if ((e = allow_lds((const void*)k_phase1_b, lds1)) != hipSuccess) return e;
  if ((e = allow_lds((const void*)k_phase2_b, lds2)) != hipSuccess) return e;
  if ((e = allow_lds((const void*)k_phase3_b, lds3)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_phase1_b, dim3(nitems), dim3(kThreads), lds1, stream, descs, items);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_phase2_b, dim3(ninst), dim3(kThreads), lds2, stream, descs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_phase3_b, dim3(nitems), dim3(kThreads), lds3, stream, descs, items);
  return hipGetLastError();
}

hipError_t launch_serial_batched(const InstDesc* descs, int ninst, size_t lds, hipStream_t stream) {
  hipError_t e;
  if ((e = allow_lds((const void*)k_serial_b, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_serial_b, dim3(ninst), dim3(kThreads), lds, stream, descs);
  return hipGetLastError();
}

}  // namespace lqr
