// Device code of the large-state path: 65..128 states, up to 64 inputs
// (the mixed-precision robot-scale workload has n = 128, m = 64). Same method
// and phases as lqr_device.h -- per segment a parametric (dual-form) backward
// sweep, the linking solve, a rebuild from the exact boundary values and the
// forward simulation (Sec. II-A) -- laid out for blocks that no longer fit the
// LDS: a 128 x 128 value Hessian alone takes 64 KiB in float and 128 KiB in
// double. Each segment's workgroup (256 threads) keeps its n x n matrices
// (P, Gamma, Psi), the stage products Y = P[B | A | c] and the eliminated
// right-hand sides in its slice of the workspace, where they stay in the L2
// cache, and feeds the matrix cores through LDS panels (bmm); the LDS also
// holds the input Hessian (FP64), its inverse factor and the vectors.
//
// Engine E: 2 = FP32 matrix cores with float accumulation and float storage
// of the products (mixed-precision mode), 1 = FP64 matrix cores and double
// storage. In both, the input Hessian R + B'PB is assembled and factored in
// FP64, the gains K, k are formed by FP64 products, and the linking solve is
// FP64.
#pragma once

#include "big_linalg.h"
#include "lqr_device.h"

namespace lqr {
namespace big {

constexpr int kLdH = 65;  // leading dimension of the input Hessian and L^{-1} in LDS

template <int E>
using Elem = typename Mfma<E>::T;  // element type of the sweep scratch

struct SweepL {
  double *H, *Linv, *ex, *p, *psi, *gc;
  int* flags;  // [0] elimination flag, [1] non-finite value gradient
};

LQR_DEV SweepL carve_lds(double* smem) {
  SweepL s;
  s.H = smem + kPanelBytes / sizeof(double);  // m x m column-major, ld kLdH (after the panels)
  s.Linv = s.H + 64 * kLdH;       // L^{-1}, column-major, ld kLdH
  s.ex = s.Linv + 64 * kLdH;      // 3 x 64 elimination exchange
  s.p = s.ex + 3 * 64;            // value gradient (n)
  s.psi = s.p + 128;              // psi (n)
  s.gc = s.psi + 128;             // Gamma' c (n), then 256 doubles of reduction space
  s.flags = reinterpret_cast<int*>(s.gc + 3 * 128);
  return s;
}

template <typename T>
struct SweepW {
  T *P, *Y, *Ga, *Gb, *Psi, *R, *Z;
};

template <typename T>
LQR_DEV SweepW<T> carve_ws(double* base, int n, int m) {
  SweepW<T> w;
  T* q = reinterpret_cast<T*>(base);
  const int nn = n * n;
  w.P = q; q += nn;
  w.Y = q; q += n * (m + n + 1);
  w.Ga = q; q += nn;
  w.Gb = q; q += nn;
  w.Psi = q; q += nn;
  w.R = q; q += m * (2 * n + 1);
  w.Z = q;
  return w;
}

// Y = P [B_t | A_t | c_t] + [0 | 0 | p]   (row-major, leading dimension m+n+1)
template <int E, typename T>
LQR_DEV void stage_y(const InstDesc& d, int t, const T* P, const double* p, T* Y) {
  const int n = d.n, m = d.m, WY = m + n + 1;
  const double* Bt = d.B + (size_t)t * n * m;
  const double* At = d.A + (size_t)t * n * n;
  const double* ct = d.c + (size_t)t * n;
  // P is symmetric: read as P' (coalesced operand loads)
  bmm1<E, true, false>(n, m, n, P, n, Bt, m, [=](int i, int j, double v) { Y[i * WY + j] = (T)v; });
  bmm1<E, true, false>(n, n, n, P, n, At, n, [=](int i, int j, double v) { Y[i * WY + m + j] = (T)v; });
  bgemv(n, n, P, n, ct, [=](int i, double v) { Y[i * WY + m + n] = (T)(v + p[i]); });
}

// H = R_t + B'Y_B (FP64, LDS, column-major); RHS[:, 0:n+1] = B'[Y_A | y_c] + [S_t | r_t];
// with Gam: RHS[:, n+1:2n+1] = B'Gam. RHS row-major with leading dimension ldr.
template <int E, typename T>
LQR_DEV void stage_h(const InstDesc& d, int t, const T* Y, const T* Gam, double* H, T* RHS, int ldr) {
  const int n = d.n, m = d.m, WY = m + n + 1;
  const double* Bt = d.B + (size_t)t * n * m;
  const double* Rt = d.R + (size_t)t * m * m;
  const double* St = d.S ? d.S + (size_t)t * m * n : nullptr;
  const double* rt = d.r + (size_t)t * m;
  bmm1<E, true, false>(m, m + n + 1, n, Bt, m, Y, WY, [=](int i, int j, double v) {
    if (j < m) {
      H[j * kLdH + i] = v + Rt[i * m + j];
    } else if (j < m + n) {
      if (St) v += St[i * n + (j - m)];
      RHS[i * ldr + (j - m)] = (T)v;
    } else {
      RHS[i * ldr + n] = (T)(v + rt[i]);
    }
  });
  if (Gam)
    bmm1<E, true, false>(m, n, n, Bt, m, Gam, n,
                         [=](int i, int j, double v) { RHS[i * ldr + n + 1 + j] = (T)v; });
}

// [P | p] <- [Q_t | q_t] + A'[Y_A | y_c] - Z_ux'[Z_ux | z_h] (lower blocks,
// mirrored), optionally also to the double outputs Pg, pg.
template <int E, typename T>
LQR_DEV void stage_value(const InstDesc& d, int t, const T* Y, const T* Z, int ldz, T* P, double* p,
                         double* Pg, double* pg, int* nonfinite) {
  const int n = d.n, m = d.m, WY = m + n + 1;
  const double* At = d.A + (size_t)t * n * n;
  const double* Qt = d.Q + (size_t)t * n * n;
  const double* qt = d.q + (size_t)t * n;
  bmm<E, true, false, true, false>(n, n + 1, n, At, n, Y + m, WY, m, Z, ldz, Z, ldz,
      [=](int i, int j, double v) {
        if (j < n) {
          if (i >= j) {
            v += 0.5 * (Qt[i * n + j] + Qt[j * n + i]);
            P[i * n + j] = (T)v;
            P[j * n + i] = (T)v;
            if (Pg) {
              Pg[i * n + j] = v;
              Pg[j * n + i] = v;
            }
          }
        } else {
          v += qt[i];
          p[i] = v;
          if (pg) pg[i] = v;
          if (!isfinite(v)) *nonfinite = 1;
        }
      },
      SkipUpper{n});
}

// Factor the input Hessian and form L^{-1} (FP64, blocked, chol_inv64); then
// Z = L^{-1} RHS (nc columns) on the engine's matrix cores.
template <int E, typename T>
LQR_DEV void stage_eliminate(int m, int nc, const SweepL& s, double* chol, const T* RHS, int ldr, T* Z) {
  chol_inv64(s.H, kLdH, m, s.Linv, kLdH, chol, s.flags);
  bmm1<E, true, false>(m, nc, m, s.Linv, kLdH, RHS, ldr,
                       [=](int i, int j, double v) { Z[i * ldr + j] = (T)v; });
}

// Plain Riccati recursion over [t0, t1) from the value (Pend, pend) at t1
// (double, global memory); writes K_t, k_t (and chol_t, P_t, p_t when
// requested). Leaves P_{t0} in the scratch (w.P) and p_{t0} in s.p. Returns a
// status code (note_pivot; LQR_INFO_NONFINITE for a non-finite gradient).
template <int E>
LQR_DEV int plain_sweep(const InstDesc& d, int t0, int t1, const double* Pend, const double* pend,
                        double* scratch, double* smem) {
  using T = Elem<E>;
  const int n = d.n, m = d.m, ldr = n + 1;
  const SweepL s = carve_lds(smem);
  const SweepW<T> w = carve_ws<T>(scratch, n, m);
  if (threadIdx.x == 0) {
    s.flags[0] = 0;
    s.flags[1] = 0;
  }
  bcopy(w.P, n, Pend, n, n, n);
  for (int i = threadIdx.x; i < n; i += nthreads()) s.p[i] = pend[i];
  __syncthreads();
  int fail = 0;
  for (int t = t1 - 1; t >= t0; --t) {
    stage_y<E>(d, t, w.P, s.p, w.Y);
    __syncthreads();
    stage_h<E>(d, t, w.Y, (const T*)nullptr, s.H, w.R, ldr);
    __syncthreads();
    stage_eliminate<E>(m, n + 1, s, d.chol ? d.chol + (size_t)t * m * m : nullptr, w.R, ldr, w.Z);
    fail = note_pivot(fail, s.flags[0], t);
    __syncthreads();
    stage_value<E>(d, t, w.Y, w.Z, ldr, w.P, s.p, d.P ? d.P + (size_t)t * n * n : nullptr,
                   d.p ? d.p + (size_t)t * n : nullptr, s.flags + 1);
    {  // [K | k] = -(L^{-1})'[Z_ux | z_h], FP64
      double* Kt = d.K + (size_t)t * m * n;
      double* kt = d.k + (size_t)t * m;
      bmm1<1, false, false>(m, n + 1, m, s.Linv, kLdH, w.Z, ldr, [=](int i, int j, double v) {
        if (j < n) Kt[i * n + j] = -v;
        else kt[i] = -v;
      });
    }
    __syncthreads();
  }
  return (fail == 0 && s.flags[1]) ? LQR_INFO_NONFINITE : fail;
}

// Parametric (dual-form) sweep of a middle segment [t0, t1), as dual_sweep in
// lqr_device.h: from P0 = 0, pbar = 0, Gam = I, Psi = 0, psi = 0, per stage
// with Z = L^{-1}[H_ux | h_u | B'Gam]:
//   P0 <- Q + A'P0A - Z_ux'Z_ux, pbar <- q + A'(P0c + pbar) - Z_ux'z_h,
//   Psi += Z_W'Z_W, psi += Gam'c - Z_W'z_h, Gam <- A'Gam - Z_ux'Z_W.
// Writes P0 | Gam | Psi | pbar | psi (double) to `out`.
template <int E>
LQR_DEV int dual_sweep(const InstDesc& d, int t0, int t1, double* out, double* scratch, double* smem) {
  using T = Elem<E>;
  const int n = d.n, m = d.m, nn = n * n, ldr = 2 * n + 1;
  const SweepL s = carve_lds(smem);
  const SweepW<T> w = carve_ws<T>(scratch, n, m);
  if (threadIdx.x == 0) {
    s.flags[0] = 0;
    s.flags[1] = 0;
  }
  bfill(w.P, n, n, n, T(0), T(0));
  bfill(w.Psi, n, n, n, T(0), T(0));
  bfill(w.Ga, n, n, n, T(0), T(1));
  for (int i = threadIdx.x; i < n; i += nthreads()) {
    s.p[i] = 0.0;
    s.psi[i] = 0.0;
  }
  __syncthreads();
  T* Gam = w.Ga;
  T* Gn = w.Gb;
  int fail = 0;
  for (int t = t1 - 1; t >= t0; --t) {
    const double* At = d.A + (size_t)t * nn;
    const double* ct = d.c + (size_t)t * n;
    stage_y<E>(d, t, w.P, s.p, w.Y);
    double* gc = s.gc;
    bgemv_t(n, n, Gam, n, ct, gc + 128, [=](int j, double v) { gc[j] = v; });  // Gam' c
    __syncthreads();
    stage_h<E>(d, t, w.Y, Gam, s.H, w.R, ldr);
    __syncthreads();
    stage_eliminate<E>(m, 2 * n + 1, s, nullptr, w.R, ldr, w.Z);
    fail = note_pivot(fail, s.flags[0], t);
    __syncthreads();
    const T* Z = w.Z;
    stage_value<E>(d, t, w.Y, Z, ldr, w.P, s.p, nullptr, nullptr, s.flags + 1);
    {  // Psi += Z_W'Z_W, psi += Gam'c - Z_W'z_h
      T* Psi = w.Psi;
      double* psi = s.psi;
      bmm1<E, true, false>(n, n + 1, m, Z + n + 1, ldr, Z + n, ldr,
          [=](int i, int j, double v) {
            if (j == 0) {
              psi[i] += gc[i] - v;
            } else if (i >= j - 1) {
              const int jj = j - 1;
              const T nv = (T)((double)Psi[i * n + jj] + v);
              Psi[i * n + jj] = nv;
              Psi[jj * n + i] = nv;
            }
          },
          SkipUpperShift{n, 1});
    }
    // Gam <- A'Gam - Z_ux'Z_W into the other buffer
    bmm<E, true, false, true, false>(n, n, n, At, n, Gam, n, m, Z, ldr, Z + n + 1, ldr,
                                     [=](int i, int j, double v) { Gn[i * n + j] = (T)v; });
    __syncthreads();
    T* tmp = Gam;
    Gam = Gn;
    Gn = tmp;
  }
  bcopy(out, n, w.P, n, n, n);
  bcopy(out + nn, n, Gam, n, n, n);
  bcopy(out + 2 * nn, n, w.Psi, n, n, n);
  for (int i = threadIdx.x; i < n; i += nthreads()) {
    out[3 * nn + i] = s.p[i];
    out[3 * nn + n + i] = s.psi[i];
  }
  return fail;
}

// Forward simulation of stages [t0, t1) from x_{t0} = xs (as rollout in
// lqr_device.h, for n <= 128, m <= 64): u_t = K_t x_t + k_t,
// x_{t+1} = A_t x_t + B_t u_t + c_t, lam_t = P_t x_t + p_t when requested.
// Eight lanes per matrix row; the state alternates between two LDS vectors.
// Returns LQR_INFO_NONFINITE (uniformly) if a value it wrote is not finite.
LQR_DEV int roll_forward(const InstDesc& d, int t0, int t1, const double* xs, bool last, double* smem) {
  const int n = d.n, m = d.m, T = d.T;
  double* sx = smem;        // two state buffers of 128
  double* su = smem + 256;  // input (64)
  int* flag = reinterpret_cast<int*>(su + 64);
  const bool want_lam = d.lam != nullptr;
  if (threadIdx.x == 0) flag[0] = 0;
  for (int i = threadIdx.x; i < n; i += nthreads()) sx[i] = xs[i];
  __syncthreads();
  int cur = 0;
  for (int t = t0; t < t1; ++t) {
    const double* x = sx + cur * 128;
    double* xn = sx + (1 - cur) * 128;
    for (int i = threadIdx.x; i < n; i += nthreads()) {
      d.x[(size_t)t * n + i] = x[i];
      if (!isfinite(x[i])) flag[0] = 1;
    }
    const double* kt = d.k + (size_t)t * m;
    bgemv(m, n, d.K + (size_t)t * m * n, n, x, [=](int i, double v) {
      const double u = v + kt[i];
      su[i] = u;
      d.u[(size_t)t * m + i] = u;
      if (!isfinite(u)) flag[0] = 1;
    });
    if (want_lam) {
      const double* pt = d.p + (size_t)t * n;
      bgemv(n, n, d.P + (size_t)t * n * n, n, x, [=](int i, double v) {
        const double l = v + pt[i];
        d.lam[(size_t)t * n + i] = l;
        if (!isfinite(l)) flag[0] = 1;
      });
    }
    __syncthreads();
    const double* At = d.A + (size_t)t * n * n;
    const double* Bt = d.B + (size_t)t * n * m;
    const double* ct = d.c + (size_t)t * n;
    {  // x' = A x + B u + c: eight lanes per row
      const int sub = threadIdx.x & 7;
      for (int i = threadIdx.x >> 3; i < n; i += nthreads() >> 3) {
        double a = 0.0;
        for (int l = sub; l < n; l += 8) a = fma(At[(size_t)i * n + l], x[l], a);
        for (int l = sub; l < m; l += 8) a = fma(Bt[(size_t)i * m + l], su[l], a);
        a += __shfl_xor(a, 1, 64);
        a += __shfl_xor(a, 2, 64);
        a += __shfl_xor(a, 4, 64);
        if (sub == 0) xn[i] = a + ct[i];
      }
    }
    __syncthreads();
    cur = 1 - cur;
  }
  if (last) {
    const double* x = sx + cur * 128;
    for (int i = threadIdx.x; i < n; i += nthreads()) {
      d.x[(size_t)T * n + i] = x[i];
      if (!isfinite(x[i])) flag[0] = 1;
    }
    if (want_lam) {
      const double* pT = d.p + (size_t)T * n;
      bgemv(n, n, d.P + (size_t)T * n * n, n, x, [=](int i, double v) {
        const double l = v + pT[i];
        d.lam[(size_t)T * n + i] = l;
        if (!isfinite(l)) flag[0] = 1;
      });
    }
  }
  __syncthreads();
  const int bad = flag[0];
  __syncthreads();
  return bad ? LQR_INFO_NONFINITE : 0;
}

// Terminal value P_T = Q_T, p_T = q_T into the outputs (if requested).
LQR_DEV void store_terminal(const InstDesc& d) {
  const int n = d.n, T = d.T;
  if (d.P) bcopy(d.P + (size_t)T * n * n, n, d.Q + (size_t)T * n * n, n, n, n);
  if (d.p)
    for (int i = threadIdx.x; i < n; i += nthreads()) d.p[(size_t)T * n + i] = d.q[(size_t)T * n + i];
}

template <int E>
LQR_DEV void phase1_item(const InstDesc& d, int seg, double* smem) {
  const int n = d.n, m = d.m, T = d.T, J = d.J;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  double* scratch = big_sweep_ws(d.ws, n, m, J, seg);
  int fail;
  if (seg < J - 1) {
    fail = dual_sweep<E>(d, t0, t1, ws_seg(d.ws, n, seg), scratch, smem);
  } else {
    store_terminal(d);
    fail = plain_sweep<E>(d, t0, t1, d.Q + (size_t)T * n * n, d.q + (size_t)T * n, scratch, smem);
    const SweepW<Elem<E>> w = carve_ws<Elem<E>>(scratch, n, m);
    const SweepL s = carve_lds(smem);
    double* b = ws_bnd(d.ws, n, J, J - 1);
    bcopy(b, n, w.P, n, n, n);
    for (int i = threadIdx.x; i < n; i += nthreads()) b[n * n + i] = s.p[i];
  }
  if (threadIdx.x == 0) d.fail[seg] = fail;
}

template <int E>
LQR_DEV void phase3_item(const InstDesc& d, int seg, double* smem) {
  const int n = d.n, m = d.m, T = d.T, J = d.J;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  if (seg < J - 1) {
    const double* b = ws_bnd(d.ws, n, J, seg + 1);
    const int fail = plain_sweep<E>(d, t0, t1, b, b + n * n, big_sweep_ws(d.ws, n, m, J, seg), smem);
    if (fail && threadIdx.x == 0) report_info(d.info, fail);
  }
  __syncthreads();
  const int nf = roll_forward(d, t0, t1, ws_bnd(d.ws, n, J, seg) + n * n + n, seg == J - 1, smem);
  if (nf && threadIdx.x == 0) report_info(d.info, nf);
}

template <int E>
LQR_DEV void serial_item(const InstDesc& d, double* smem) {
  const int n = d.n, m = d.m, T = d.T;
  store_terminal(d);
  const int fail = plain_sweep<E>(d, 0, T, d.Q + (size_t)T * n * n, d.q + (size_t)T * n,
                                  big_sweep_ws(d.ws, n, m, 1, 0), smem);
  __syncthreads();
  const int nf = roll_forward(d, 0, T, d.x0, true, smem);
  if (threadIdx.x == 0) *d.info = combine_info(fail, nf);
}

}  // namespace big
}  // namespace lqr
