// Plain Riccati recursion (Sec. II, eqs. Kx, k1, update:Vxx, update:vx) for
// instances with n <= 16 and m <= 16, one 256-thread workgroup per instance.
//
// At these sizes a stage is a few thousand multiply-adds and the general sweep
// is bound by latency: global loads on the dependency chain and barriers per
// pivot. Here every block lives in LDS padded to 16 x 16 with zeros, so that
// thread (i, j) = (tid / 16, tid % 16) owns one element of each 16 x 16
// product and no loop depends on n or m; the next stage's inputs are loaded
// into registers at the top of a stage and stored to the other half of a
// double buffer at its end, so their latency overlaps the stage's work. A
// stage costs four barriers:
//   1. Y = P A, W = P B (matrix cores), g = P c + p        (waves 0-2)
//   2. H = R + B'W, Hux = S + B'Y (matrix cores), h = r + B'g (waves 0-2)
//   3. H = L_unit D L_unit', [K | k] = -H^{-1}[Hux | h]   (wave 0, see below)
//      and meanwhile Q + A'Y, q + A'g                     (waves 1-3)
//   4. P <- (Q + A'Y) + Hux'K, p <- (q + A'g) + Hux'k     (all threads)
// Loops carry no lane-dependent branches (every thread runs the same dot
// products and only the stores are conditional), so no LDS wait lands inside
// a loop. Thread (i, j) of a symmetric result computes element
// (max(i, j), min(i, j)) in a fixed order, so both halves are bitwise equal.
// The forward simulation (x, u, costates) uses the same layout and staging,
// with the state's whole chain in one wave.
#include "lqr_device.h"
#include "lqr_kernels.h"
#include "lqr_launch.h"

namespace lqr {

namespace {

constexpr int kS = 16;            // padded block edge
constexpr int kB = kS * kS;       // padded block size
// one half of the stage-input double buffer: A | B | S | Q | R | c | q | r
constexpr int kStageDoubles = 5 * kB + 3 * kS;
// LDS carve (doubles): 2 stage buffers, then P | p | Y | W | g | H | Hux | h |
// K | kv | Lu | Pa | pa | D | zero, then (dual form) Gam | W | X | A'Gam |
// Psi[2] | psi | Gam'c, then two int flags
constexpr int kSmallDoubles = 2 * kStageDoubles + 14 * kB + 11 * kS;

struct StageRegs {
  double a, b, s, q2, r2, v;  // this thread's element of A, B, S, Q, R; of c, q or r
};

// This thread's share of stage t's inputs (zero outside the instance's sizes).
LQR_DEV StageRegs fetch_stage(const InstDesc& d, int t, int i, int j) {
  const int n = d.n, m = d.m;
  StageRegs g;
  g.a = (i < n && j < n) ? gp(d.A)[(size_t)t * n * n + i * n + j] : 0.0;
  g.b = (i < n && j < m) ? gp(d.B)[(size_t)t * n * m + i * m + j] : 0.0;
  g.s = (d.S && i < m && j < n) ? gp(d.S)[(size_t)t * m * n + i * n + j] : 0.0;
  g.q2 = (i < n && j < n) ? gp(d.Q)[(size_t)t * n * n + i * n + j] : 0.0;
  g.r2 = (i < m && j < m) ? gp(d.R)[(size_t)t * m * m + i * m + j] : 0.0;
  g.v = 0.0;
  if (j == 0 && i < n) g.v = gp(d.c)[(size_t)t * n + i];
  if (j == 1 && i < n) g.v = gp(d.q)[(size_t)t * n + i];
  if (j == 2 && i < m) g.v = gp(d.r)[(size_t)t * m + i];
  return g;
}

// Forward simulation at these sizes: one half of its double buffer holds
// P | K | A | B | k | p | c of a stage.
constexpr int kRollDoubles = 4 * kB + 3 * kS;

// This thread's share of stage t's simulation data: K, A, B, k, c when t is
// a stage of the range (t < t1), P and p when costates are requested.
LQR_DEV StageRegs fetch_roll(const InstDesc& d, int t, bool st, int i, int j) {
  const int n = d.n, m = d.m;
  const bool lam = d.lam != nullptr;
  StageRegs g;
  g.a = (lam && i < n && j < n) ? gp(d.P)[(size_t)t * n * n + i * n + j] : 0.0;
  g.b = (st && i < m && j < n) ? gp(d.K)[(size_t)t * m * n + i * n + j] : 0.0;
  g.s = (st && i < n && j < n) ? gp(d.A)[(size_t)t * n * n + i * n + j] : 0.0;
  g.q2 = (st && i < n && j < m) ? gp(d.B)[(size_t)t * n * m + i * m + j] : 0.0;
  g.r2 = 0.0;
  g.v = 0.0;
  if (st && j == 0 && i < m) g.v = gp(d.k)[(size_t)t * m + i];
  if (lam && j == 1 && i < n) g.v = gp(d.p)[(size_t)t * n + i];
  if (st && j == 2 && i < n) g.v = gp(d.c)[(size_t)t * n + i];
  return g;
}

LQR_DEV void store_roll(double* buf, const StageRegs& g, int i, int j) {
  const int e = i * kS + j;
  buf[e] = g.a;
  buf[kB + e] = g.b;
  buf[2 * kB + e] = g.s;
  buf[3 * kB + e] = g.q2;
  if (j < 3) buf[4 * kB + j * kS + i] = g.v;
}

// Forward simulation of stages [t0, t1) from x_{t0} = xs (global):
// u_t = K_t x_t + k_t, x_{t+1} = A_t x_t + B_t u_t + c_t, lam_t = P_t x_t + p_t
// (when requested); writes x_t, u_t, lam_t and, if last, x_{t1} and
// lam_{t1}. The whole chain of a stage stays in wave 0 (lane r holds x_r and
// u_r; the other lanes' values come by readlane), so a stage costs one
// workgroup barrier: wave 1 forms the costate from the state in LDS while
// every thread stages the next stage's blocks. Returns LQR_INFO_NONFINITE
// (uniformly) if any value written is not finite, else 0.
LQR_DEV int rollout_small(const InstDesc& d, int t0, int t1, const double* xs, bool last,
                          double* smem) {
  const int n = d.n, m = d.m;
  const int tid = threadIdx.x, i = tid >> 4, j = tid & 15, lane = tid & 63, r = lane & 15;
  const bool want_lam = d.lam != nullptr;
  double* sx = smem + 2 * kRollDoubles;  // [2][16]: x_t by stage parity
  int* anybad = reinterpret_cast<int*>(sx + 2 * kS);
  bool finite = true;
  double x = r < n ? gp(xs)[r] : 0.0;  // wave 0's state, lane r
  if (tid < kS) sx[tid] = x;
  store_roll(smem, fetch_roll(d, t0, t0 < t1, i, j), i, j);
  __syncthreads();
  int cur = 0;
  for (int t = t0; t < t1; ++t, cur ^= 1) {
    const double* bP = smem + cur * kRollDoubles;
    const double* bK = bP + kB;
    const double* bA = bP + 2 * kB;
    const double* bB = bP + 3 * kB;
    const double* bk = bP + 4 * kB;
    const double* bp = bk + kS;
    const double* bc = bp + kS;
    const StageRegs next = fetch_roll(d, t + 1, t + 1 < t1, i, j);
    if (tid < 64) {
      if (lane < n) {
        gp(d.x)[(size_t)t * n + lane] = x;
        finite = finite && isfinite(x);
      }
      double u = bk[r], xn = bc[r];
      static_for<0, kS>([&](auto L) {
        constexpr int l = decltype(L)::value;
        const double xl = readlane(x, l);
        u = fma(bK[r * kS + l], xl, u);
        xn = fma(bA[r * kS + l], xl, xn);
      });
      if (lane < m) {
        gp(d.u)[(size_t)t * m + lane] = u;
        finite = finite && isfinite(u);
      }
      static_for<0, kS>([&](auto L) {
        constexpr int l = decltype(L)::value;
        xn = fma(bB[r * kS + l], readlane(u, l), xn);
      });
      x = xn;
      if (lane < kS) sx[((t + 1 - t0) & 1) * kS + lane] = x;
    } else if (tid < 128 && want_lam) {
      const double* xt = sx + ((t - t0) & 1) * kS;
      double v = bp[r];
#pragma unroll 8
      for (int l = 0; l < kS; ++l) v = fma(bP[r * kS + l], xt[l], v);
      if (lane < n) {
        gp(d.lam)[(size_t)t * n + lane] = v;
        finite = finite && isfinite(v);
      }
    }
    store_roll(smem + (cur ^ 1) * kRollDoubles, next, i, j);
    __syncthreads();
  }
  if (last) {
    if (tid < 64 && lane < n) {
      gp(d.x)[(size_t)t1 * n + lane] = x;
      finite = finite && isfinite(x);
    } else if (tid >= 64 && tid < 128 && want_lam) {
      const double* bP = smem + cur * kRollDoubles;
      const double* bp = bP + 4 * kB + kS;
      const double* xt = sx + ((t1 - t0) & 1) * kS;
      double v = bp[r];
#pragma unroll 8
      for (int l = 0; l < kS; ++l) v = fma(bP[r * kS + l], xt[l], v);
      if (lane < n) {
        gp(d.lam)[(size_t)t1 * n + lane] = v;
        finite = finite && isfinite(v);
      }
    }
  }
  const int wave = tid >> 6;
  const bool wbad = __ballot(!finite) != 0ull;
  if (lane == 0) anybad[wave] = wbad ? 1 : 0;
  __syncthreads();
  int bad = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) bad |= anybad[w];
  __syncthreads();
  return bad ? LQR_INFO_NONFINITE : 0;
}

LQR_DEV void store_stage(double* buf, const StageRegs& g, int i, int j) {
  const int e = i * kS + j;
  buf[e] = g.a;
  buf[kB + e] = g.b;
  buf[2 * kB + e] = g.s;
  buf[3 * kB + e] = g.q2;
  buf[4 * kB + e] = g.r2;
  if (j < 3) buf[5 * kB + j * kS + i] = g.v;
}

// Rounds of the L_unit D L_unit' elimination and the back substitution for a
// fixed m = M (wave 0; lane c holds column c of [H | Hux | h]): the pivot and
// the entries H(r, k), r > k, come from lane k by readlane, so the chain
// touches no LDS; the multipliers go to Lu for the back substitution and the
// pivots to D. bad: as note_pivot expects.
template <int M>
LQR_DEV void ldl_rounds(double (&v)[kS], int c, int& bad, double* sLu, double* sD) {
  static_for<0, M>([&](auto Kc) {
    constexpr int k = decltype(Kc)::value;
    double dk = readlane(v[k], k);
    if (!(dk > 0.0) || !isfinite(dk)) {
      if (!bad) bad = isfinite(dk) ? 1 : 2;
      dk = __builtin_nan("");
    }
    const double tk = v[k] * recip(dk);
    if (c > k && c < M) sLu[c * kS + k] = tk;
    if (c == 0) sD[k] = dk;
    static_for<k + 1, M>([&](auto I) {
      constexpr int r = decltype(I)::value;
      v[r] = fma(-readlane(v[r], k), tk, v[r]);
    });
    v[k] = tk;
  });
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  static_for<1, M>([&](auto Ic) {
    constexpr int r = M - decltype(Ic)::value;  // M-1 .. 1
    const double xr = v[r];
    static_for<0, r>([&](auto Kc) {
      constexpr int k = decltype(Kc)::value;
      v[k] = fma(-sLu[r * kS + k], xr, v[k]);
    });
  });
}

template <int... Ms>
LQR_DEV void ldl_dispatch(int m, double (&v)[kS], int c, int& bad, double* sLu, double* sD) {
  ((m == Ms ? (ldl_rounds<Ms>(v, c, bad, sLu, sD), 0) : 0), ...);
}

}  // namespace

// Plain recursion over stages [t0, t1) from the value (Pend, pend) at t1
// (global memory, symmetrised on load); writes K, k, P, p, chol for those
// stages. With DUAL, the parametric (dual-form) sweep of a segment instead:
// the value starts at zero with Gam = I, Psi = 0, psi = 0 at t1, and per stage,
// with W = B'Gam (the old Gam) and X = H^{-1} W from the same elimination as
// the gains,
//   Psi += W'X,  psi += Gam'c + W'k,  Gam <- A'Gam + K'W,
// no per-stage output is written, and P0 | Gam | Psi | pbar | psi go to `out`
// at the end. Returns a status code as note_pivot builds it
// (LQR_INFO_NONFINITE also for a non-finite value gradient), uniform over
// the workgroup. Ends with a barrier; smem may be reused afterwards.
template <bool DUAL>
LQR_DEV int small_sweep(const InstDesc& d, int t0, int t1, const double* Pend, const double* pend,
                        double* out, double* smem) {
  const int n = d.n, m = d.m;
  const int tid = threadIdx.x, i = tid >> 4, j = tid & 15;
  double* sP = smem + 2 * kStageDoubles;
  double* sp = sP + kB;
  double* sY = sp + kS;
  double* sW = sY + kB;
  double* sg = sW + kB;
  double* sH = sg + kS;
  double* sHux = sH + kB;
  double* sh = sHux + kB;
  double* sK = sh + kS;
  double* skv = sK + kB;
  double* sLu = skv + kS;     // unit lower factor of H (row-major, below the diagonal)
  double* sPa = sLu + kB;     // Q + A'Y
  double* spa = sPa + kB;     // q + A'g
  double* sD = spa + kS;      // pivots of H, then their square roots
  double* sZero = sD + kS;    // 16 zeros
  double* sGam = sZero + kS;  // Gam (dual form)
  double* sWg = sGam + kB;    // W = B'Gam
  double* sXg = sWg + kB;     // X = H^{-1} W
  double* sAG = sXg + kB;     // A'Gam
  double* sPsi = sAG + kB;    // [2]: Psi, ping-pong across stages
  double* spsi = sPsi + 2 * kB;
  double* sGc = spsi + kS;    // Gam'c
  int* flags = reinterpret_cast<int*>(DUAL ? sGc + kS : sZero + kS);  // [0]: non-finite value gradient
  const int mx = i > j ? i : j, mn = i > j ? j : i;

  // value at t1, the last stage's inputs, zero gains (rows >= m stay zero)
  if (DUAL) {
    sP[tid] = 0.0;
    if (tid < kS) sp[tid] = 0.0;
    sGam[tid] = (i == j && i < n) ? 1.0 : 0.0;
    sPsi[tid] = 0.0;
    if (tid < kS) spsi[tid] = 0.0;
  } else {
    sP[tid] = (i < n && j < n) ? 0.5 * (gp(Pend)[i * n + j] + gp(Pend)[j * n + i]) : 0.0;
    if (tid < kS) sp[tid] = tid < n ? gp(pend)[tid] : 0.0;
  }
  sK[tid] = 0.0;
  if (tid < kS) {
    skv[tid] = 0.0;
    sZero[tid] = 0.0;
  }
  if (tid == 0) flags[0] = 0;
  store_stage(smem, fetch_stage(d, t1 - 1, i, j), i, j);
  __syncthreads();

  int fail = 0;  // wave 0's status (note_pivot)
  for (int t = t1 - 1, cur = 0; t >= t0; --t, cur ^= 1) {
    const double* sPsiOld = sPsi + cur * kB;  // DUAL: this stage's Psi in, the other half out
    double* sPsiNew = sPsi + (cur ^ 1) * kB;
    const double* bA = smem + cur * kStageDoubles;
    const double* bB = bA + kB;
    const double* bS = bA + 2 * kB;
    const double* bQ = bA + 3 * kB;
    const double* bR = bA + 4 * kB;
    const double* bc = bA + 5 * kB;
    const double* bq = bc + kS;
    const double* br = bq + kS;
    const StageRegs next = fetch_stage(d, t > t0 ? t - 1 : t0, i, j);

    // 1. Y = P A (wave 0) and W = P B (wave 1) on the matrix cores, g = P c + p
    //    (wave 2). P is exactly symmetric, so its column k is read as row k.
    {
      const int wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
      if (wv < 2) {
        const double* Yop = wv == 0 ? bA : bB;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + lk;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sP[k * kS + li], Yop[k * kS + li], acc, 0, 0, 0);
        }
        double* out = wv == 0 ? sY : sW;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(lk + 4 * r) * kS + li] = acc[r];
      } else if (wv == 2 && lane < kS) {
        double gc = sp[lane];
#pragma unroll 8
        for (int l = 0; l < kS; ++l) gc = fma(sP[l * kS + lane], bc[l], gc);
        sg[lane] = gc;
      } else if (DUAL && wv == 3 && lane < kS) {
        double gc = 0.0;
#pragma unroll 8
        for (int l = 0; l < kS; ++l) gc = fma(sGam[l * kS + lane], bc[l], gc);
        sGc[lane] = gc;
      }
    }
    __syncthreads();

    // 2. H = R + B'W (symmetrised R; wave 0) and Hux = S + B'Y (wave 1) on the
    //    matrix cores, h = r + B'g (wave 2)
    {
      const int wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
      if (wv < 2) {
        f64x4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = lk + 4 * r;
          acc[r] = wv == 0 ? 0.5 * (bR[ii * kS + li] + bR[li * kS + ii]) : bS[ii * kS + li];
        }
        const double* Yop = wv == 0 ? sW : sY;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + lk;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bB[k * kS + li], Yop[k * kS + li], acc, 0, 0, 0);
        }
        double* out = wv == 0 ? sH : sHux;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(lk + 4 * r) * kS + li] = acc[r];
      } else if (DUAL && wv == 2) {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + lk;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bB[k * kS + li], sGam[k * kS + li], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sWg[(lk + 4 * r) * kS + li] = acc[r];
      } else if (wv == (DUAL ? 3 : 2) && lane < kS) {
        double hv = br[lane];
#pragma unroll 8
        for (int l = 0; l < kS; ++l) hv = fma(bB[l * kS + lane], sg[l], hv);
        sh[lane] = hv;
      }
    }
    __syncthreads();

    // 3. Wave 0: lane c < m holds column c of H, lane m + c (c < n) column c
    //    of Hux, lane m + n the vector h, other lanes zeros; rows >= m are
    //    zero and stay zero. Round k reads the pivot d_k = H(k, k) and
    //    H(r, k), r > k, from lane k (readlane; the rounds are unrolled for the
    //    instance's m), and every lane updates its column,
    //    v_r -= H(r, k) (v_k / d_k) for r > k. The trailing block stays
    //    symmetric, so lane c > k's v_k / d_k is the unit lower factor's entry
    //    (c, k), kept in Lu, and v_k / d_k is also the right-hand side's entry
    //    of D^{-1} L_unit^{-1} [Hux | h]. Back substitution with L_unit' then
    //    gives H^{-1}[Hux | h] = -[K | k], left in LDS (rows >= m zero); the
    //    square roots of the pivots for the Cholesky factor L = L_unit D^{1/2}
    //    go to D. Step 4 writes K, k and L to global memory.
    if (tid < 64) {
      const int c = tid;
      const bool rcol = c >= m && c < m + n, vcol = c == m + n;
      const bool wcol = DUAL && c > m + n && c <= m + 2 * n;  // columns of W (dual form)
      const double* col = c < m ? sH + c : rcol ? sHux + (c - m) : vcol ? sh
                                        : wcol ? sWg + (c - m - n - 1) : sZero;
      const int cs = (c < m || rcol || wcol) ? kS : 1;
      double v[kS];
      static_for<0, kS>([&](auto R) { v[decltype(R)::value] = col[decltype(R)::value * cs]; });
      int bad = 0;
      ldl_dispatch<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16>(m, v, c, bad, sLu, sD);
      if (rcol) {
        static_for<0, kS>([&](auto Kc) { sK[decltype(Kc)::value * kS + (c - m)] = -v[decltype(Kc)::value]; });
      } else if (vcol) {
        static_for<0, kS>([&](auto Kc) { skv[decltype(Kc)::value] = -v[decltype(Kc)::value]; });
      } else if (wcol) {
        static_for<0, kS>([&](auto Kc) { sXg[decltype(Kc)::value * kS + (c - m - n - 1)] = v[decltype(Kc)::value]; });
      }
      fail = note_pivot(fail, bad, t);
      if (c < m) sD[c] = sqrt(sD[c]);
    } else {
      // waves 1-3: the parts of the new value that do not need the gains
      for (int e = tid - 64; e < kB; e += kThreads - 64) {
        const int ei = e >> 4, ej = e & 15;
        const int ex = ei > ej ? ei : ej, en = ei > ej ? ej : ei;
        double v = 0.5 * (bQ[ei * kS + ej] + bQ[ej * kS + ei]);
#pragma unroll 8
        for (int l = 0; l < kS; ++l) v = fma(bA[l * kS + ex], sY[l * kS + en], v);
        sPa[e] = v;
      }
      if (tid < 64 + kS) {
        const int r = tid - 64;
        double v = bq[r];
#pragma unroll 8
        for (int l = 0; l < kS; ++l) v = fma(bA[l * kS + r], sg[l], v);
        spa[r] = v;
      }
      if (DUAL && tid >= 192) {
        const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + lk;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bA[k * kS + li], sGam[k * kS + li], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sAG[(lk + 4 * r) * kS + li] = acc[r];
      }
    }
    __syncthreads();

    // 4. P <- (Q + A'Y) + Hux'K, p <- (q + A'g) + Hux'k; the next stage's
    //    inputs go to the other buffer
    {
      double v = sPa[mx * kS + mn];
#pragma unroll 8
      for (int l = 0; l < kS; ++l) v = fma(sHux[l * kS + mx], sK[l * kS + mn], v);
      sP[tid] = v;
      if (!DUAL && d.P && i < n && j < n) gp(d.P)[(size_t)t * n * n + i * n + j] = v;
      if (tid < kS) {
        double w = spa[tid];
#pragma unroll 8
        for (int l = 0; l < kS; ++l) w = fma(sHux[l * kS + tid], skv[l], w);
        sp[tid] = w;
        if (tid < n) {
          if (!DUAL && d.p) gp(d.p)[(size_t)t * n + tid] = w;
          if (!isfinite(w)) flags[0] = 1;
        }
      }
      if (DUAL) {
        // Psi += W'X (element (max, min), so the halves stay bitwise equal),
        // Gam <- A'Gam + K'W, psi += Gam'c + W'k
        double ps = sPsiOld[mx * kS + mn], ga = sAG[tid];
#pragma unroll 8
        for (int l = 0; l < kS; ++l) {
          ps = fma(sWg[l * kS + mx], sXg[l * kS + mn], ps);
          ga = fma(sK[l * kS + i], sWg[l * kS + j], ga);
        }
        sPsiNew[tid] = ps;
        sGam[tid] = ga;
        if (tid >= 64 && tid < 64 + kS) {
          const int r = tid - 64;
          double w = spsi[r] + sGc[r];
#pragma unroll 8
          for (int l = 0; l < kS; ++l) w = fma(sWg[l * kS + r], skv[l], w);
          spsi[r] = w;
        }
      } else {
        // gains and Cholesky factor of this stage, from LDS (coalesced)
        if (i < m && j < n) gp(d.K)[(size_t)t * m * n + i * n + j] = sK[tid];
        if (tid < m) gp(d.k)[(size_t)t * m + tid] = skv[tid];
        if (d.chol && i < m && j < m)
          gp(d.chol)[(size_t)t * m * m + i * m + j] = j < i ? sLu[i * kS + j] * sD[j] : j == i ? sD[i] : 0.0;
      }
      if (t > t0) store_stage(smem + (cur ^ 1) * kStageDoubles, next, i, j);
    }
    __syncthreads();
  }
  if (DUAL && i < n && j < n) {  // the segment's summary, row-major n x n blocks
    const int nn = n * n, e = i * n + j;
    const double* psiF = sPsi + ((t1 - t0) & 1) * kB;  // the half the last stage wrote
    gp(out)[e] = sP[tid];
    gp(out)[nn + e] = sGam[tid];
    gp(out)[2 * nn + e] = psiF[tid];
    if (j == 0) {
      gp(out)[3 * nn + i] = sp[i];
      gp(out)[3 * nn + n + i] = spsi[i];
    }
  } else if (!DUAL && out && i < n && j < n) {  // the value at t0: P | p
    gp(out)[i * n + j] = sP[tid];
    if (j == 0) gp(out)[n * n + i] = sp[i];
  }
  const int nonfinite_p = flags[0];
  // wave 0's status to every thread
  if (tid == 0) flags[1] = (fail == 0 && nonfinite_p) ? LQR_INFO_NONFINITE : fail;
  __syncthreads();
  const int code = flags[1];
  __syncthreads();
  return code;
}

__global__ __launch_bounds__(kThreads, 2) void k_small_serial(InstDesc single, const InstDesc* descs,
                                                               int spread_rollout) {
  extern __shared__ double smem[];
  const InstDesc d = descs ? descs[blockIdx.x] : single;
  const int n = d.n, T = d.T;
  write_terminal(d);
  const int sweep = small_sweep<false>(d, 0, T, d.Q + (size_t)T * n * n, d.q + (size_t)T * n, nullptr, smem);
  // with a workgroup or more per compute unit the general forward simulation,
  // which spreads each product over the four waves, keeps the SIMDs busier;
  // alone on a unit the one-wave chain has the shorter stage
  const int nf = spread_rollout ? rollout(d, 0, T, d.x0, true, smem)
                                : rollout_small(d, 0, T, d.x0, true, smem);
  if (threadIdx.x == 0) *d.info = combine_info(sweep, nf);
}

// Phase 1 of the segmented solve at these sizes, one workgroup per segment:
// the parametric sweep of segment j < J - 1 into its summary; the last
// segment's plain recursion from the terminal cost, its value at its start
// into the boundary slot. Each segment's status goes to its failure word.
__global__ __launch_bounds__(kThreads, 2) void k_small_phase1(InstDesc d) {
  extern __shared__ double smem[];
  const int n = d.n, T = d.T, J = d.J, seg = blockIdx.x;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  int fail;
  if (seg < J - 1) {
    fail = small_sweep<true>(d, t0, t1, nullptr, nullptr, ws_seg(d.ws, n, seg), smem);
  } else {
    write_terminal(d);
    fail = small_sweep<false>(d, t0, t1, d.Q + (size_t)T * n * n, d.q + (size_t)T * n,
                              ws_bnd(d.ws, n, J, J - 1), smem);
  }
  if (threadIdx.x == 0) {
    d.fail[seg] = fail;
    if (seg == 0) d.fail[J] = 0;  // the linking-failure word, raised by phase 2
  }
}

// Phase 3 of the segmented solve at these sizes, one workgroup per segment:
// the rebuild of segment j < J - 1 from the exact value at its end (the
// linking solve's boundary slot), then the forward simulation from its
// boundary state (the last segment was swept in phase 1).
__global__ __launch_bounds__(kThreads, 2) void k_small_phase3(InstDesc d) {
  extern __shared__ double smem[];
  const int n = d.n, T = d.T, J = d.J, seg = blockIdx.x;
  const int t0 = seg_begin(T, J, seg), t1 = seg_begin(T, J, seg + 1);
  if (seg < J - 1) {
    const double* b = ws_bnd(d.ws, n, J, seg + 1);
    const int fail = small_sweep<false>(d, t0, t1, b, b + n * n, nullptr, smem);
    if (fail && threadIdx.x == 0) report_info(d.info, fail);
  }
  const int nf = rollout_small(d, t0, t1, ws_bnd(d.ws, n, J, seg) + n * n + n, seg == J - 1, smem);
  if (nf && threadIdx.x == 0) report_info(d.info, nf);
}

size_t small_serial_lds() {
  const size_t sweep = kSmallDoubles * sizeof(double) + 64;
  size_t roll = (2 * kRollDoubles + 2 * kS) * sizeof(double) + 64;
  if (roll < rollout_lds(16, 16)) roll = rollout_lds(16, 16);
  return sweep > roll ? sweep : roll;
}

hipError_t launch_small_phase1(const InstDesc& d, hipStream_t stream) {
  const size_t lds = small_serial_lds();
  hipError_t e = ensure_dynamic_lds((const void*)k_small_phase1, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_small_phase1, dim3(d.J), dim3(kThreads), lds, stream, d);
  return hipGetLastError();
}

hipError_t launch_small_phase3(const InstDesc& d, hipStream_t stream) {
  const size_t lds = small_serial_lds();
  hipError_t e = ensure_dynamic_lds((const void*)k_small_phase3, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_small_phase3, dim3(d.J), dim3(kThreads), lds, stream, d);
  return hipGetLastError();
}

hipError_t launch_small_serial(const InstDesc& single, const InstDesc* descs, int ninst,
                               hipStream_t stream) {
  const size_t lds = small_serial_lds();
  hipError_t e = ensure_dynamic_lds((const void*)k_small_serial, lds);
  if (e != hipSuccess) return e;
  // 256 compute units: from one instance per unit on, spread the rollout
  hipLaunchKernelGGL(k_small_serial, dim3(ninst), dim3(kThreads), lds, stream, single, descs,
                     ninst >= 256 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace lqr
