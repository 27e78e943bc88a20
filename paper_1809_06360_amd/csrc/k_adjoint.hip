// Adjoint (gradient) of the LQR solve, FP64.
//
// The optimal (x, u, lam) solves the KKT system of eq. (KKT), whose matrix is
// symmetric; differentiating it shows that the gradient of a loss l(x, u)
// needs one more solve of the same system against the right-hand side
// dl/d(x, u): the same LQR with linear terms qhat = -dl/dx, rhat = -dl/du,
// zero offsets and a zero initial state. Its quadratic data are unchanged, so
// the forward solve's gains K_t, value Hessians P_t and Cholesky factors L_t of
// the input Hessians are reused: backward,
//   hhat_t = rhat_t + B_t' phat_{t+1},   khat_t = -(L_t L_t')^{-1} hhat_t,
//   phat_t = qhat_t + A_t' phat_{t+1} + K_t' hhat_t,   phat_T = qhat_T
// (K_t' hhat = H_ux' khat since K = -H_uu^{-1} H_ux), then forward from
// xhat_0 = 0: uhat_t = K_t xhat_t + khat_t, xhat_{t+1} = A_t xhat_t + B_t uhat_t,
// lamhat_t = P_t xhat_t + phat_t. The gradients are outer products of the two
// solutions (see k_adjoint_grad).
#include "lqr_device.h"
#include "lqr_kernels.h"
#include "lqr_launch.h"

namespace lqr {

namespace {

// Solve (L L') y = b in place for one m-vector b in LDS, L row-major (m x m,
// lower) in LDS; run by wave 0 (lane = row), m sequential steps per triangle
// with wave-level ordering only.
LQR_DEV void chol_solve_wave(const double* L, int m, double* b) {
  const int lane = threadIdx.x & 63;
  for (int k = 0; k < m; ++k) {  // L z = b
    const double zk = b[k] / L[k * m + k];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) b[k] = zk;
    if (lane > k && lane < m) b[lane] = fma(-L[lane * m + k], zk, b[lane]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  for (int k = m - 1; k >= 0; --k) {  // L' y = z
    const double yk = b[k] / L[k * m + k];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) b[k] = yk;
    if (lane < k) b[lane] = fma(-L[k * m + lane], yk, b[lane]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------
// n, m <= 16: blocks zero-padded to 16 x 16 in a double-buffered LDS area.
// Thread (i, j) = (tid / 16, tid % 16) loads element (i, j) of the next
// stage's blocks into registers at the top of a stage and stores them into
// the other buffer at its end, so no global load sits on the recursion's
// chain. The substitutions with the Cholesky factor run in registers of
// wave 0 (lane r holds row r; the pivot value comes by readlane).
// ---------------------------------------------------------------------------
constexpr int kAS = 16, kAB = kAS * kAS;
// one buffer: four blocks and two vectors
constexpr int kAdjBuf = 4 * kAB + 2 * kAS;
constexpr int kAdjSmallDoubles = 2 * kAdjBuf + 7 * kAS;

struct AdjRegs {
  double b0, b1, b2, b3, v;
};

// Backward stage t: A, B, K, L and (j == 0) qhat_t = -dl/dx_t, (j == 1)
// rhat_t = -dl/du_t.
LQR_DEV AdjRegs fetch_back(const AdjDesc& a, int t, int i, int j) {
  const int n = a.n, m = a.m;
  AdjRegs g;
  g.b0 = (i < n && j < n) ? gp(a.A)[(size_t)t * n * n + i * n + j] : 0.0;
  g.b1 = (i < n && j < m) ? gp(a.B)[(size_t)t * n * m + i * m + j] : 0.0;
  g.b2 = (i < m && j < n) ? gp(a.K)[(size_t)t * m * n + i * n + j] : 0.0;
  g.b3 = (i < m && j < m) ? gp(a.chol)[(size_t)t * m * m + i * m + j] : 0.0;
  g.v = 0.0;
  if (j == 0 && i < n) g.v = -gp(a.dl_dx)[(size_t)t * n + i];
  if (j == 1 && i < m) g.v = -gp(a.dl_du)[(size_t)t * m + i];
  return g;
}

// Forward stage t: P, K, A, B and (j == 0) khat_t, (j == 1) phat_t.
LQR_DEV AdjRegs fetch_fwd(const AdjDesc& a, const double* kh, const double* ph, int t, int i, int j) {
  const int n = a.n, m = a.m, T = a.T;
  AdjRegs g;
  g.b0 = (i < n && j < n) ? gp(a.P)[(size_t)t * n * n + i * n + j] : 0.0;
  const bool st = t < T;  // stage T has only P and phat
  g.b1 = (st && i < m && j < n) ? gp(a.K)[(size_t)t * m * n + i * n + j] : 0.0;
  g.b2 = (st && i < n && j < n) ? gp(a.A)[(size_t)t * n * n + i * n + j] : 0.0;
  g.b3 = (st && i < n && j < m) ? gp(a.B)[(size_t)t * n * m + i * m + j] : 0.0;
  g.v = 0.0;
  if (st && j == 0 && i < m) g.v = gp(kh)[(size_t)t * m + i];
  if (j == 1 && i < n) g.v = gp(ph)[(size_t)t * n + i];
  return g;
}

LQR_DEV void store_regs(double* buf, const AdjRegs& g, int i, int j) {
  const int e = i * kAS + j;
  buf[e] = g.b0;
  buf[kAB + e] = g.b1;
  buf[2 * kAB + e] = g.b2;
  buf[3 * kAB + e] = g.b3;
  if (j < 2) buf[4 * kAB + j * kAS + i] = g.v;
}

// (L L') y = b for lane r holding b_r (rows >= M zero), unrolled for m = M:
// the substituted values come from their lanes by readlane and the
// reciprocals of L's diagonal from rd, so the chain has no LDS wait or guard.
template <int M>
LQR_DEV double chol_solve_lanes(double y, int r, const double* L, const double* rd) {
  static_for<0, M>([&](auto Kc) {
    constexpr int k = decltype(Kc)::value;
    const double zk = readlane(y, k) * rd[k];
    y = r == k ? zk : (r > k ? fma(-L[r * kAS + k], zk, y) : y);
  });
  static_for<0, M>([&](auto Kc) {
    constexpr int k = M - 1 - decltype(Kc)::value;
    const double yk = readlane(y, k) * rd[k];
    y = r == k ? yk : (r < k ? fma(-L[k * kAS + r], yk, y) : y);
  });
  return y;
}

template <int... Ms>
LQR_DEV double chol_solve_dispatch(int m, double y, int r, const double* L, const double* rd) {
  ((m == Ms ? (y = chol_solve_lanes<Ms>(y, r, L, rd), 0) : 0), ...);
  return y;
}

LQR_DEV void adjoint_small(const AdjDesc& a, double* smem) {
  const int n = a.n, m = a.m, T = a.T;
  const int tid = threadIdx.x, i = tid >> 4, j = tid & 15, lane = tid & 63;
  double* ph = a.ws;
  double* kh = ph + (size_t)(T + 1) * n;
  double* xh = kh + (size_t)T * m;
  double* uh = xh + (size_t)(T + 1) * n;
  double* lh = uh + (size_t)T * m;
  double* sv = smem + 2 * kAdjBuf;
  double* sp = sv;            // phat_{t+1}
  double* sh = sp + kAS;      // hhat_t
  double* sacc = sh + kAS;    // qhat_t + A_t' phat_{t+1}
  double* sx0 = sacc + kAS;   // xhat (ping-pong with sx1)
  double* sx1 = sx0 + kAS;
  double* sspare = sx1 + kAS; // (spare)
  double* srd = sspare + kAS; // 1 / L_t(k, k)

  // backward. Wave 0 forms hhat in registers and runs the substitutions with
  // it; wave 1 forms hhat again (sixteen products) and then phat, so the two
  // need no exchange and a stage costs one barrier. phat alternates between
  // two LDS vectors by stage parity (wave 0 reads the old one while wave 1
  // writes the new one).
  double* sp0 = sp;
  double* sp1 = sacc;
  if (tid < kAS) {
    const double v = tid < n ? -gp(a.dl_dx)[(size_t)T * n + tid] : 0.0;
    sp0[tid] = v;
    if (tid < n) gp(ph)[(size_t)T * n + tid] = v;
  }
  store_regs(smem, fetch_back(a, T - 1, i, j), i, j);
  __syncthreads();
  for (int t = T - 1, cur = 0; t >= 0; --t, cur ^= 1) {
    const double* bA = smem + cur * kAdjBuf;
    const double* bB = bA + kAB;
    const double* bK = bA + 2 * kAB;
    const double* bL = bA + 3 * kAB;
    const double* bq = bA + 4 * kAB;
    const double* br = bq + kAS;
    const double* spo = ((T - 1 - t) & 1) ? sp1 : sp0;  // phat_{t+1}
    double* spn = ((T - 1 - t) & 1) ? sp0 : sp1;        // phat_t
    const AdjRegs next = fetch_back(a, t > 0 ? t - 1 : 0, i, j);
    if (tid < 128) {
      const int r = lane & 15;
      double hv = br[r];  // hhat = rhat + B' phat
#pragma unroll 8
      for (int l = 0; l < kAS; ++l) hv = fma(bB[l * kAS + r], spo[l], hv);
      if (tid < 64) {
        // (L L') y = hhat: lane r holds y_r; rows >= m are zero
        const double rd = r < m ? 1.0 / bL[r * kAS + r] : 0.0;
        if (lane < kAS) srd[lane] = rd;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double y = chol_solve_dispatch<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16>(
            m, hv, r, bL, srd);
        if (lane < m) gp(kh)[(size_t)t * m + lane] = -y;
      } else {
        // phat_t = qhat + A' phat + K' hhat
        double v = bq[r];
#pragma unroll 8
        for (int l = 0; l < kAS; ++l) v = fma(bA[l * kAS + r], spo[l], v);
        static_for<0, kAS>([&](auto L) {
          constexpr int l = decltype(L)::value;
          v = fma(bK[l * kAS + r], readlane(hv, l), v);
        });
        if (lane < kAS) spn[lane] = v;
        if (lane < n) gp(ph)[(size_t)t * n + lane] = v;
      }
    }
    if (t > 0) store_regs(smem + (cur ^ 1) * kAdjBuf, next, i, j);
    __syncthreads();
  }
  // forward from xhat_0 = 0. The state's chain stays in wave 0 (lane r holds
  // xhat_r and uhat_r, the other lanes' values by readlane), so a stage costs
  // one barrier; wave 1 forms lamhat from the state in LDS (by stage parity).
  if (tid < kAS) sx0[tid] = 0.0;
  store_regs(smem, fetch_fwd(a, kh, ph, 0, i, j), i, j);
  __syncthreads();
  double x = 0.0;  // wave 0: xhat_t of row lane & 15
  for (int t = 0, cur = 0; t <= T; ++t, cur ^= 1) {
    const double* bP = smem + cur * kAdjBuf;
    const double* bK = bP + kAB;
    const double* bA = bP + 2 * kAB;
    const double* bB = bP + 3 * kAB;
    const double* bk = bP + 4 * kAB;
    const double* bp = bk + kAS;
    const double* sx = (t & 1) ? sx1 : sx0;
    double* sxn = (t & 1) ? sx0 : sx1;
    const AdjRegs next = fetch_fwd(a, kh, ph, t < T ? t + 1 : T, i, j);
    if (tid < 64) {
      const int r = lane & 15;
      if (lane < n) gp(xh)[(size_t)t * n + lane] = x;
      if (t < T) {
        double u = bk[r], xn = 0.0;
        static_for<0, kAS>([&](auto L) {
          constexpr int l = decltype(L)::value;
          const double xl = readlane(x, l);
          u = fma(bK[r * kAS + l], xl, u);
          xn = fma(bA[r * kAS + l], xl, xn);
        });
        if (lane < m) gp(uh)[(size_t)t * m + lane] = u;
        static_for<0, kAS>([&](auto L) {
          constexpr int l = decltype(L)::value;
          xn = fma(bB[r * kAS + l], readlane(u, l), xn);
        });
        x = xn;
        if (lane < kAS) sxn[lane] = x;
      }
    } else if (tid < 128) {
      const int r = lane & 15;
      double v = bp[r];
#pragma unroll 8
      for (int l = 0; l < kAS; ++l) v = fma(bP[r * kAS + l], sx[l], v);
      if (lane < n) gp(lh)[(size_t)t * n + lane] = v;
    }
    if (t == T) break;
    store_regs(smem + (cur ^ 1) * kAdjBuf, next, i, j);
    __syncthreads();
  }
}

}  // namespace

size_t adjoint_small_lds() { return (size_t)kAdjSmallDoubles * sizeof(double) + 64; }

// One workgroup per instance: the adjoint backward and forward recursions.
// Workspace per instance (AdjDesc::ws): phat (T+1)n | khat T m | xhat (T+1)n |
// uhat T m | lamhat (T+1)n.
__global__ __launch_bounds__(kThreads) void k_adjoint_solve(const AdjDesc* descs) {
  extern __shared__ double smem[];
  const AdjDesc a = descs[blockIdx.x];
  const int n = a.n, m = a.m, T = a.T;
  if (n <= kAS && m <= kAS) {
    adjoint_small(a, smem);
    return;
  }
  double* ph = a.ws;
  double* kh = ph + (size_t)(T + 1) * n;
  double* xh = kh + (size_t)T * m;
  double* uh = xh + (size_t)(T + 1) * n;
  double* lh = uh + (size_t)T * m;
  double* sp = smem;      // phat_{t+1} (n)
  double* sh = sp + n;    // hhat (m), then khat
  double* sh2 = sh + m;   // copy of hhat for K' hhat
  double* sx = sh2 + m;   // xhat_t (n)
  double* sxn = sx + n;   // xhat_{t+1} (n)
  double* su = sxn + n;   // uhat_t (m)
  double* sL = su + m;    // Cholesky factor of stage t's input Hessian (m x m)

  for (int i = threadIdx.x; i < n; i += kThreads) {
    const double v = -a.dl_dx[(size_t)T * n + i];
    sp[i] = v;
    ph[(size_t)T * n + i] = v;
  }
  __syncthreads();
  for (int t = T - 1; t >= 0; --t) {
    const LQR_GLOBAL double* At = gp(a.A + (size_t)t * n * n);
    const LQR_GLOBAL double* Bt = gp(a.B + (size_t)t * n * m);
    const LQR_GLOBAL double* Kt = gp(a.K + (size_t)t * m * n);
    // the factor to LDS, so that the substitutions' chain of 2m dependent
    // steps reads no global memory
    const LQR_GLOBAL double* Lt = gp(a.chol + (size_t)t * m * m);
    for (int e = threadIdx.x; e < m * m; e += kThreads) sL[e] = Lt[e];
    // hhat = rhat + B' phat  (column i of B against phat)
    for (int i = threadIdx.x; i < m; i += kThreads) {
      double s = -gp(a.dl_du)[(size_t)t * m + i];
      for (int l = 0; l < n; ++l) s = fma(Bt[l * m + i], sp[l], s);
      sh[i] = s;
      sh2[i] = s;
    }
    __syncthreads();
    // phat_t = qhat + A' phat + K' hhat   (reads sp, sh2; written below after a barrier)
    double acc = 0.0;
    const int i = threadIdx.x;
    if (i < n) {
      acc = -gp(a.dl_dx)[(size_t)t * n + i];
      for (int l = 0; l < n; ++l) acc = fma(At[l * n + i], sp[l], acc);
      for (int l = 0; l < m; ++l) acc = fma(Kt[l * n + i], sh2[l], acc);
    }
    if (threadIdx.x < 64) chol_solve_wave(sL, m, sh);
    __syncthreads();
    if (i < n) {
      sp[i] = acc;
      gp(ph)[(size_t)t * n + i] = acc;
    }
    for (int j = threadIdx.x; j < m; j += kThreads) gp(kh)[(size_t)t * m + j] = -sh[j];
    __syncthreads();
  }
  // forward: xhat_0 = 0
  for (int j = threadIdx.x; j < n; j += kThreads) sx[j] = 0.0;
  __syncthreads();
  for (int t = 0; t <= T; ++t) {
    const double* Pt = a.P + (size_t)t * n * n;
    double* xo = xh + (size_t)t * n;
    double* lo = lh + (size_t)t * n;
    for (int j = threadIdx.x; j < n; j += kThreads) xo[j] = sx[j];
    gemv2(n, n, Pt, n, sx, 0, sx, 0, sx,
          [=](int r, double v) { lo[r] = ph[(size_t)t * n + r] + v; });
    if (t == T) break;
    const double* At = a.A + (size_t)t * n * n;
    const double* Bt = a.B + (size_t)t * n * m;
    const double* Kt = a.K + (size_t)t * m * n;
    gemv2(m, n, Kt, n, sx, 0, sx, 0, sx, [=](int r, double v) {
      v += kh[(size_t)t * m + r];
      su[r] = v;
      uh[(size_t)t * m + r] = v;
    });
    __syncthreads();
    gemv2(n, n, At, n, sx, m, Bt, m, su, [=](int r, double v) { sxn[r] = v; });
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kThreads) sx[j] = sxn[j];
    __syncthreads();
  }
}

// Gradient outer products, one workgroup per (instance, block of stages):
//   dq_t = -xhat_t, dr_t = -uhat_t, dc_t = -lamhat_{t+1}, dx0 = -lamhat_0,
//   dQ_t = -(xhat_t x_t' + x_t xhat_t')/2, dR_t = -(uhat_t u_t' + u_t uhat_t')/2,
//   dS_t = -(uhat_t x_t' + u_t xhat_t'),
//   dA_t = -(lamhat_{t+1} x_t' + lam_{t+1} xhat_t'),
//   dB_t = -(lamhat_{t+1} u_t' + lam_{t+1} uhat_t').
// Every output element is written by exactly one thread with coalesced rows.
// The block's vectors (x, xhat, u, uhat, lam_{t+1}, lamhat_{t+1} of each of its
// stages) are first copied to LDS in one pass, so the stores of the outer
// products wait for one round of loads rather than one per stage.
constexpr int kGradVec = 4 * 128 + 2 * 64;  // per stage, at the largest n and m

__global__ __launch_bounds__(kThreads) void k_adjoint_grad(const AdjDesc* descs, const int2* blocks) {
  extern __shared__ double sv[];  // kAdjStages x kGradVec (dynamic, like every kernel's LDS)
  const int2 bk = blocks[blockIdx.x];
  const AdjDesc a = descs[bk.x];
  const int n = a.n, m = a.m, T = a.T;
  const double* ph = a.ws;
  const double* xh = ph + (size_t)(T + 1) * n + (size_t)T * m;
  const double* uh = xh + (size_t)(T + 1) * n;
  const double* lh = uh + (size_t)T * m;
  const int t0 = bk.y * kAdjStages, t1 = min(T + 1, t0 + kAdjStages);
  // per stage: x | xhat | lam_{t+1} | lamhat_{t+1} (n each) | u | uhat (m each)
  const int vs = 4 * n + 2 * m;
  for (int e = threadIdx.x; e < (t1 - t0) * vs; e += kThreads) {
    const int s = e / vs, q = e - s * vs, t = t0 + s;
    double v = 0.0;
    if (q < n) v = gp(a.x)[(size_t)t * n + q];
    else if (q < 2 * n) v = gp(xh)[(size_t)t * n + (q - n)];
    else if (t < T && q < 3 * n) v = gp(a.lam)[(size_t)(t + 1) * n + (q - 2 * n)];
    else if (t < T && q < 4 * n) v = gp(lh)[(size_t)(t + 1) * n + (q - 3 * n)];
    else if (t < T && q < 4 * n + m) v = gp(a.u)[(size_t)t * m + (q - 4 * n)];
    else if (t < T && q >= 4 * n + m) v = gp(uh)[(size_t)t * m + (q - 4 * n - m)];
    sv[s * kGradVec + q] = v;
  }
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    const double* sx = sv + (t - t0) * kGradVec;
    const double* xt = sx;
    const double* xht = sx + n;
    if (a.dq)
      for (int i = threadIdx.x; i < n; i += kThreads) gp(a.dq)[(size_t)t * n + i] = -xht[i];
    if (a.dQ)
      for (int e = threadIdx.x; e < n * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        gp(a.dQ)[(size_t)t * n * n + e] = -0.5 * (xht[i] * xt[j] + xt[i] * xht[j]);
      }
    if (t == 0 && a.dx0)
      for (int i = threadIdx.x; i < n; i += kThreads) gp(a.dx0)[i] = -gp(lh)[i];
    if (t == T) continue;
    const double* ut = sx + 4 * n;
    const double* uht = sx + 4 * n + m;
    const double* l1 = sx + 2 * n;
    const double* lh1 = sx + 3 * n;
    if (a.dr)
      for (int i = threadIdx.x; i < m; i += kThreads) gp(a.dr)[(size_t)t * m + i] = -uht[i];
    if (a.dc)
      for (int i = threadIdx.x; i < n; i += kThreads) gp(a.dc)[(size_t)t * n + i] = -lh1[i];
    if (a.dR)
      for (int e = threadIdx.x; e < m * m; e += kThreads) {
        const int i = e / m, j = e - i * m;
        gp(a.dR)[(size_t)t * m * m + e] = -0.5 * (uht[i] * ut[j] + ut[i] * uht[j]);
      }
    if (a.dS)
      for (int e = threadIdx.x; e < m * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        gp(a.dS)[(size_t)t * m * n + e] = -(uht[i] * xt[j] + ut[i] * xht[j]);
      }
    if (a.dA)
      for (int e = threadIdx.x; e < n * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        gp(a.dA)[(size_t)t * n * n + e] = -(lh1[i] * xt[j] + l1[i] * xht[j]);
      }
    if (a.dB)
      for (int e = threadIdx.x; e < n * m; e += kThreads) {
        const int i = e / m, j = e - i * m;
        gp(a.dB)[(size_t)t * n * m + e] = -(lh1[i] * ut[j] + l1[i] * uht[j]);
      }
  }
}

hipError_t launch_adjoint(const AdjDesc* descs, int ninst, const int2* blocks, int nblocks,
                          size_t lds, hipStream_t stream) {
  hipError_t e = ensure_dynamic_lds((const void*)k_adjoint_solve, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adjoint_solve, dim3(ninst), dim3(kThreads), lds, stream, descs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t glds = (size_t)kAdjStages * kGradVec * sizeof(double);
  if ((e = ensure_dynamic_lds((const void*)k_adjoint_grad, glds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_adjoint_grad, dim3(nblocks), dim3(kThreads), glds, stream, descs, blocks);
  return hipGetLastError();
}

}  // namespace lqr
