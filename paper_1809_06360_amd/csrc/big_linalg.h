// Workgroup linear algebra of the large-state kernels (65..128 states, up to
// 64 inputs), for gfx950.
//
// Operands are generic pointers (LDS or global memory, float or double): the
// matrices of a 128-state stage do not fit the LDS together, so most of them
// live in the workspace and are read through the L2 cache. Every routine is
// called by all threads of the workgroup with identical arguments and does
// not synchronise at its end.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lqr_layout.h"
#include "wg_linalg.h"

namespace lqr {
namespace big {

// Workgroup sizes: the linking kernels run 512 threads (8 wave64s, two per
// SIMD; the register-resident Gauss-Jordan inverse needs all of them), the
// sweep kernels 256 (one wave per SIMD with the full register file: their FP64
// elimination keeps a 64-row column per lane). The routines below work for
// either size (they read blockDim.x).
constexpr int kBT = 512;
constexpr int kSweepThreads = 256;

LQR_DEV int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
LQR_DEV int nthreads() { return __builtin_amdgcn_readfirstlane(blockDim.x); }
LQR_DEV int nwaves() { return nthreads() >> 6; }

// Matrix-core instruction of a product engine: E = 1 FP64 (16x16x4 f64),
// E = 2 FP32 (16x16x4 f32, operands rounded to float, float accumulation).
template <int E> struct Mfma;
template <> struct Mfma<1> {
  using T = double;
  using V = f64x4;
  static LQR_DEV V op(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // row of result register r in lane group g (column = lane % 16)
  static LQR_DEV int row(int g, int r) { return g + 4 * r; }
};
template <> struct Mfma<2> {
  using T = float;
  using V = f32x4;
  static LQR_DEV V op(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static LQR_DEV int row(int g, int r) { return 4 * g + r; }
};

// ---------------------------------------------------------------------------
// Matrix-core product of the large-state kernels, staged through LDS:
//   v(i, j) = sum_k op(A1)(i,k) op(B1)(k,j) - sum_k op(A2)(i,k) op(B2)(k,j)
// for 0 <= i < M <= 128, 0 <= j < N, handed to epi(i, j, v) (v widened to
// double). The output is produced in strips of 128 columns; for each strip
// the k range (K1, then K2 with the sign flipped) is walked in panels of KP:
// all threads load the A panel (M x KP) and the B panel (KP x 128) with
// coalesced global loads (consecutive threads read consecutive addresses),
// convert them to the engine's precision and store them in LDS; each wave
// then runs the MFMAs of its 32 x 32 output blocks (2 x 2 tiles of 16 x 16)
// from LDS. Panels are double-buffered: the global loads of panel p+1 are
// issued before the MFMAs of panel p, so their latency is hidden behind the
// matrix-core work. `skip(i0, j0, 32, 32)` may drop output blocks.
//
// The two panel buffers occupy the first kPanelBytes of the workgroup's
// dynamic LDS; callers keep their own LDS data after that. Must be called by
// every thread of a workgroup of NT threads; ends with a barrier.
// ---------------------------------------------------------------------------
template <int E>
struct Panel {
  static constexpr int KP = E == 2 ? 32 : 16;    // k per panel
  static constexpr int LDA = KP + 1;             // A panel: 128 x KP (padded)
  static constexpr int LDB = 132;                // B panel: KP x 128 (padded)
  static constexpr int ELEMS = 128 * LDA + KP * LDB;
};
constexpr size_t kPanelBytes = 2 * (size_t)Panel<1>::ELEMS * sizeof(double);
static_assert(2 * Panel<2>::ELEMS * sizeof(float) <= kPanelBytes, "panel buffers");
static_assert(kPanelBytes == kBigPanelBytes, "planner's LDS budget");

// Panel element r of thread t. Consecutive threads read consecutive memory
// for the operand's storage order: the thread's elements share one coordinate
// (`fixed`) and step the other by a constant (`base + r * STEP`), so a load's
// address is a base pointer plus a fixed increment per element and little
// index state stays in registers. Wide: the panel's 128-long coordinate is the
// contiguous one in memory (then it is the fixed one, t % 128).
//   A panel (128 rows i x KP columns kk), Wide = TA (A stored as A[k * lda + i]);
//   B panel (KP rows kk x 128 columns j), Wide = !TB (B stored as B[k * ldb + j]).
template <int KP, int NT, bool Wide>
struct PanelWalk {
  static constexpr int STEP = Wide ? NT / 128 : NT / KP;
  static LQR_DEV int fixed(int t) { return Wide ? (t & 127) : (t % KP); }
  static LQR_DEV int base(int t) { return Wide ? (t >> 7) : (t / KP); }
};

template <int E, bool TA1, bool TB1, bool TA2, bool TB2, int NT = kSweepThreads, typename PA1,
          typename PB1, typename PA2, typename PB2, typename Epi, typename Skip = NoSkip>
LQR_DEV void bmm(int M, int N, int K1, const PA1* A1, int lda1, const PB1* B1, int ldb1, int K2,
                 const PA2* A2, int lda2, const PB2* B2, int ldb2, Epi epi, Skip skip = Skip()) {
  using T = typename Mfma<E>::T;
  using V = typename Mfma<E>::V;
  using PL = Panel<E>;
  constexpr int KP = PL::KP, LDA = PL::LDA, LDB = PL::LDB;
  constexpr int NW = NT / 64;
  constexpr int QB = (16 + NW - 1) / NW;       // output blocks per wave and strip (at most)
  constexpr int RL = 128 * KP / NT;            // panel elements per thread and operand
  extern __shared__ double lds_dyn[];
  T* const pan = reinterpret_cast<T*>(lds_dyn);
  // The thread index passes through an empty asm: every per-thread index and
  // address below is then computed inside this call, not hoisted out of the
  // callers' loops where the addresses of all their products would stay live.
  int t = threadIdx.x;
  __asm__ volatile("" : "+v"(t));
  const int lane = t & 63, wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int np1 = (K1 + KP - 1) / KP, np = np1 + (K2 + KP - 1) / KP;
  if (np == 0 || M <= 0 || N <= 0) return;
  for (int n0 = 0; n0 < N; n0 += 128) {
    const int ns = min(128, N - n0);
    const int nbj = (ns + 31) >> 5, nb = ((M + 31) >> 5) * nbj;
    T ra[RL], rb[RL];
    // global loads of panel p of one product into ra (A: 128 x KP), rb (B: KP x 128)
    auto gload_part = [&](auto tag, int k0) {
      constexpr bool FIRST = decltype(tag)::value;
      using WA = PanelWalk<KP, NT, FIRST ? TA1 : TA2>;
      using WB = PanelWalk<KP, NT, !(FIRST ? TB1 : TB2)>;
      constexpr bool TA = FIRST ? TA1 : TA2, TB = FIRST ? TB1 : TB2;
      const int K = FIRST ? K1 : K2;
      const T sg = FIRST ? T(1) : T(-1);
      // The leading dimensions pass through an empty asm so that the compiler
      // does not hoist the RL element addresses of every product out of the
      // callers' loops (they would pin hundreds of registers).
      int lda = FIRST ? lda1 : lda2, ldb = FIRST ? ldb1 : ldb2;
      __asm__ volatile("" : "+s"(lda), "+s"(ldb));
      const int af = WA::fixed(t), ab = WA::base(t);
      const int bf = WB::fixed(t), bb = WB::base(t);
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int av = ab + r * WA::STEP, bv = bb + r * WB::STEP;
        const int i = TA ? af : av, ka = k0 + (TA ? av : af);
        const int kb = k0 + (TB ? bf : bv), j = n0 + (TB ? bv : bf);
        const bool oka = i < M && ka < K, okb = kb < K && j - n0 < ns;
        const int ic = oka ? i : 0, kac = oka ? ka : 0, kbc = okb ? kb : 0, jc = okb ? j : 0;
        T va, vb;
        if constexpr (FIRST) {
          va = (T)el<TA1>(A1, lda, ic, kac);
          vb = (T)el<TB1>(B1, ldb, kbc, jc);
        } else {
          va = (T)el<TA2>(A2, lda, ic, kac);
          vb = (T)el<TB2>(B2, ldb, kbc, jc);
        }
        ra[r] = oka ? sg * va : T(0);
        rb[r] = okb ? vb : T(0);
      }
    };
    auto gload = [&](int p) {
      if (p < np1) gload_part(std::true_type{}, p * KP);
      else gload_part(std::false_type{}, (p - np1) * KP);
    };
    auto lstore_part = [&](auto tag, int buf) {
      constexpr bool FIRST = decltype(tag)::value;
      using WA = PanelWalk<KP, NT, FIRST ? TA1 : TA2>;
      using WB = PanelWalk<KP, NT, !(FIRST ? TB1 : TB2)>;
      constexpr bool TA = FIRST ? TA1 : TA2, TB = FIRST ? TB1 : TB2;
      T* Ap = pan + buf * PL::ELEMS;
      T* Bp = Ap + 128 * LDA;
      const int af = WA::fixed(t), ab = WA::base(t);
      const int bf = WB::fixed(t), bb = WB::base(t);
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int av = ab + r * WA::STEP, bv = bb + r * WB::STEP;
        const int i = TA ? af : av, kk = TA ? av : af;
        const int kb = TB ? bf : bv, j = TB ? bv : bf;
        Ap[i * LDA + kk] = ra[r];
        Bp[kb * LDB + j] = rb[r];
      }
    };
    auto lstore = [&](int p, int buf) {
      if (p < np1) lstore_part(std::true_type{}, buf);
      else lstore_part(std::false_type{}, buf);
    };
    gload(0);
    lstore(0, 0);
    V acc[QB][2][2];
#pragma unroll
    for (int q = 0; q < QB; ++q)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[q][u][v] = V{};
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      if (p + 1 < np) gload(p + 1);
      const T* Ap = pan + (p & 1) * PL::ELEMS;
      const T* Bp = Ap + 128 * LDA;
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int blk = wave + q * NW;
        const int i0 = (blk / nbj) << 5, j0 = (blk % nbj) << 5;
        if (blk >= nb || skip(i0, n0 + j0, 32, 32)) continue;
#pragma unroll
        for (int s4 = 0; s4 < KP / 4; ++s4) {
          T a[2], b[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            a[u] = Ap[(i0 + 16 * u + li) * LDA + 4 * s4 + lk];
            b[u] = Bp[(4 * s4 + lk) * LDB + j0 + 16 * u + li];
          }
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) acc[q][u][v] = Mfma<E>::op(a[u], b[v], acc[q][u][v]);
        }
      }
      if (p + 1 < np) lstore(p + 1, (p + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int blk = wave + q * NW;
      const int i0 = (blk / nbj) << 5, j0 = (blk % nbj) << 5;
      if (blk >= nb || skip(i0, n0 + j0, 32, 32)) continue;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * u + Mfma<E>::row(lk, r), j = j0 + 16 * v + li;
            if (i < M && j < ns) epi(i, n0 + j, (double)acc[q][u][v][r]);
          }
    }
  }
}

template <int E, bool TA, bool TB, int NT = kSweepThreads, typename PA, typename PB, typename Epi,
          typename Skip = NoSkip>
LQR_DEV void bmm1(int M, int N, int K, const PA* A, int lda, const PB* B, int ldb, Epi epi,
                  Skip skip = Skip()) {
  bmm<E, TA, TB, false, false, NT>(M, N, K, A, lda, B, ldb, 0, A, lda, B, ldb, epi, skip);
}

// y(i) = epi(i, sum_l M[i][l] v[l]) for i < rows (M row-major, any memory; v
// in LDS or global). Eight lanes per row, each summing every eighth column with
// eight loads in flight, then a reduction over the eight lanes.
template <typename PM, typename PV, typename Epi>
LQR_DEV void bgemv(int rows, int cols, const PM* Mx, int ld, const PV* v, Epi epi) {
  const int sub = threadIdx.x & 7;
  // the eight lanes of a row share i, so each shuffle group is fully active
  for (int i = threadIdx.x >> 3; i < rows; i += nthreads() >> 3) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < cols; l0 += 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int l = l0 + sub + 8 * u;
        if (l < cols) a[u & 3] = fma((double)Mx[(size_t)i * ld + l], (double)v[l], a[u & 3]);
      }
    }
    double s = (a[0] + a[1]) + (a[2] + a[3]);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    if (sub == 0) epi(i, s);
  }
}

// y(j) = epi(j, sum_l M[l][j] v[l]) for j < cols <= 128: the transposed
// product. Thread t takes column t % 128 and every G-th row (G = threads /
// 128), with eight rows in flight (coalesced: consecutive threads read
// consecutive columns of a row); the G partial sums meet in `red` (LDS,
// nthreads doubles). Ends with a barrier.
template <typename PM, typename PV, typename Epi>
LQR_DEV void bgemv_t(int rows, int cols, const PM* Mx, int ld, const PV* v, double* red, Epi epi) {
  const int t = threadIdx.x, j = t & 127, g = t >> 7, G = nthreads() >> 7;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (j < cols) {
    int l = g;
    for (; l + 7 * G < rows; l += 8 * G) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = fma((double)Mx[(size_t)(l + u * G) * ld + j], (double)v[l + u * G], acc[u]);
    }
    for (; l < rows; l += G) acc[0] = fma((double)Mx[(size_t)l * ld + j], (double)v[l], acc[0]);
  }
  red[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (t < cols) {
    double sum = 0.0;
    for (int h = 0; h < G; ++h) sum += red[h * 128 + t];
    epi(t, sum);
  }
  __syncthreads();
}

// Copy rows x cols between any memories with conversion (dst leading ldd).
template <typename D, typename S>
LQR_DEV void bcopy(D* dst, int ldd, const S* src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += nthreads()) {
    const int i = e / cols, j = e - i * cols;
    dst[(size_t)i * ldd + j] = (D)src[(size_t)i * lds + j];
  }
}

template <typename D>
LQR_DEV void bfill(D* dst, int ldd, int rows, int cols, D v, D diag) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += nthreads()) {
    const int i = e / cols, j = e - i * cols;
    dst[(size_t)i * ldd + j] = (i == j) ? diag : v;
  }
}

// ---------------------------------------------------------------------------
// Cholesky factorization H = L L' of an m x m symmetric positive definite
// matrix (m <= 64, FP64) and the inverse of its factor, blocked by 16 and
// right-looking, with all threads of the workgroup:
//  1. diagonal block: wave 0 factors it column-owner style (lane c holds
//     column c, pivots read across lanes), and lanes 16..31 carry the
//     identity as right-hand sides, which take the same row operations, so
//     the block's L_kk^{-1} comes out of the same pass;
//  2. panel: L_ik = H_ik L_kk^{-T}, one thread per row below the block;
//  3. trailing update of the lower triangle: H_ij -= L_ik L_jk';
// then the off-diagonal blocks of L^{-1}, block row by block row,
//  X_ij = -L_ii^{-1} sum_{k=j}^{i-1} L_ik X_kj.
// H: column-major in LDS (element (i, j) at H[j * ldh + i]); only its lower
// triangle is read; on return it holds L in the lower triangle. Linv:
// column-major (ld ldl) receives L^{-1} with zeros above the diagonal. chol
// (optional, any memory): L row-major, zeros above the diagonal. A pivot that
// is not positive or not finite is replaced by NaN and *flag set to 1 (first
// failing pivot finite: not positive definite) or 2 (not finite), as
// ldl_columns does. Requires a barrier between H's producer and this call;
// ends with a barrier.
// ---------------------------------------------------------------------------
LQR_DEV void chol_inv64(double* H, int ldh, int m, double* Linv, int ldl, double* chol, int* flag) {
  const int t = threadIdx.x, nt = nthreads(), lane = t & 63, wave = wave_id();
  const int nb = (m + 15) >> 4;
  int badf = 0;
  for (int kb = 0; kb < nb; ++kb) {
    const int c0 = kb * 16, bs = min(16, m - c0);
    if (wave == 0) {
      const bool isH = lane < bs, isR = lane >= 16 && lane - 16 < bs;
      const int q = lane - 16;
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double h = 0.0;
        if (isH && i < bs) h = i >= lane ? H[(c0 + lane) * ldh + c0 + i] : H[(c0 + i) * ldh + c0 + lane];
        v[i] = isH ? h : ((isR && i == q) ? 1.0 : 0.0);
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < bs) {
          double dk = readlane(v[k], k);
          if (!(dk > 0.0) || !isfinite(dk)) {
            if (!badf) badf = isfinite(dk) ? 1 : 2;
            dk = qnan<double>();
          }
          const double sk = (isR || (isH && lane > k)) ? v[k] / dk : 0.0;
#pragma unroll
          for (int i = k + 1; i < 16; ++i) v[i] = fma(-readlane(v[i], k), sk, v[i]);
        }
      }
      double dc = v[0];
#pragma unroll
      for (int i = 1; i < 16; ++i)
        if (i == lane) dc = v[i];
      if (!(dc > 0.0) || !isfinite(dc)) dc = qnan<double>();
      const double sc = sqrt(dc), rs = 1.0 / sc;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double ri = readlane(rs, i);
        if (isR) v[i] *= ri;
      }
      if (isH) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i < bs && i >= lane) H[(c0 + lane) * ldh + c0 + i] = i == lane ? sc : v[i] * rs;
      }
      if (isR) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i < bs) Linv[(c0 + q) * ldl + c0 + i] = i >= q ? v[i] : 0.0;
      }
      if (badf && lane == 0) *flag = badf;
    }
    __syncthreads();
    const int r0 = c0 + bs, nr = m - r0;
    // panel: row r0 + i of L_ik = (row of H_ik) L_kk^{-T}
    for (int i = t; i < nr; i += nt) {
      double h[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) h[k] = k < bs ? H[(c0 + k) * ldh + r0 + i] : 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (c < bs) {
          double a = 0.0;
#pragma unroll
          for (int k = 0; k <= c; ++k) a = fma(h[k], Linv[(c0 + k) * ldl + c0 + c], a);
          H[(c0 + c) * ldh + r0 + i] = a;
        }
      }
    }
    __syncthreads();
    // trailing lower triangle: H(i, j) -= sum_c L(i, c) L(j, c), r0 <= j <= i < m
    for (int e = t; e < nr * nr; e += nt) {
      const int j = e / nr, i = e - j * nr;
      if (j > i) continue;
      double a = H[(r0 + j) * ldh + r0 + i];
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < bs) a = fma(-H[(c0 + c) * ldh + r0 + i], H[(c0 + c) * ldh + r0 + j], a);
      H[(r0 + j) * ldh + r0 + i] = a;
    }
    __syncthreads();
  }
  // off-diagonal blocks of L^{-1}: block row ib from the rows above it
  for (int ib = 1; ib < nb; ++ib) {
    const int i0 = ib * 16, bi = min(16, m - i0);
    for (int e = t; e < bi * i0; e += nt) {
      const int r = e % bi, j = e / bi;
      double a = 0.0;
      for (int k = j; k < i0; ++k) a = fma(H[k * ldh + i0 + r], Linv[j * ldl + k], a);
      Linv[j * ldl + i0 + r] = a;  // sum_k L_ik X_kj, finished below
    }
    __syncthreads();
    for (int j = t; j < i0; j += nt) {
      double tv[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) tv[r] = r < bi ? Linv[j * ldl + i0 + r] : 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r < bi) {
          double a = 0.0;
#pragma unroll
          for (int s2 = 0; s2 <= r; ++s2) a = fma(Linv[(i0 + s2) * ldl + i0 + r], tv[s2], a);
          Linv[j * ldl + i0 + r] = -a;
        }
      }
    }
    __syncthreads();
  }
  for (int e = t; e < m * m; e += nt) {
    const int j = e / m, i = e - j * m;
    if ((j >> 4) > (i >> 4)) Linv[j * ldl + i] = 0.0;  // blocks above the diagonal
    if (chol) chol[i * m + j] = j <= i ? H[j * ldh + i] : 0.0;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// In-place inverse of an n x n matrix (n <= 128) by Gauss-Jordan elimination
// (512-thread workgroups only)
// with partial pivoting, FP64, the matrix held in registers: thread t owns
// rows 4 (t / 16) .. +3 and columns 8 (t % 16) .. +7. Pivots are chosen
// without moving rows (pivot of column k: the unused row with the largest
// magnitude in column k, ties to the lowest row); after all n pivots the
// registers hold the inverse with its rows and columns permuted, which the
// write-back undoes. Per pivot: the owners of column k publish it, every wave
// finds the pivot row, its owners publish it, and every thread updates its 32
// elements (two barriers, double-buffered exchange vectors).
//
// Mx: n x n row-major in any memory (leading dimension ld), replaced by its
// inverse.
// xb: 4 * 128 doubles of LDS exchange space; rowof: 256 ints of LDS. A zero
// or non-finite pivot sets *bad = 1 (the result is then not meaningful).
// Requires a barrier between Mx's producer and this call; ends with a barrier.
// ---------------------------------------------------------------------------
LQR_DEV void gj_invert(double* Mx, int ld, int n, double* xb, int* rowof, int* bad) {
  const int t = threadIdx.x;
  const int r0 = (t >> 4) * 4, c0 = (t & 15) * 8;
  const int lane = t & 63;
  double v[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = r0 + a, j = c0 + b;
      v[a][b] = (i < n && j < n) ? Mx[i * ld + j] : (i == j ? 1.0 : 0.0);
    }
  uint64_t used0 = 0, used1 = 0;  // rows already pivoted (wave-uniform)
  for (int k = 0; k < n; ++k) {
    double* col = xb + (k & 1) * 256;  // column k, then row p
    double* row = col + 128;
    if (k >= c0 && k < c0 + 8) {
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if (c0 + b == k) {
#pragma unroll
          for (int a = 0; a < 4; ++a) col[r0 + a] = v[a][b];
        }
    }
    __syncthreads();
    // pivot row: every wave, rows lane and lane + 64; key = |value| bits with
    // the low 7 mantissa bits replaced by (127 - row): larger magnitude wins,
    // ties go to the lower row, NaN/inf sort first
    long long key = -1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      const bool free_row = i < n && !(((h ? used1 : used0) >> lane) & 1ull);
      if (free_row) {
        double av = fabs(col[i]);
        if (!(av <= 1.7976931348623157e308)) av = __builtin_inf();
        const long long kk =
            (long long)((__builtin_bit_cast(unsigned long long, av) & ~127ull) | (unsigned)(127 - i));
        key = kk > key ? kk : key;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const long long o = __shfl_xor(key, off, 64);
      key = o > key ? o : key;
    }
    const int p = __builtin_amdgcn_readfirstlane(127 - (int)(key & 127));
    if (p < 64) used0 |= 1ull << p; else used1 |= 1ull << (p - 64);
    if (p >= r0 && p < r0 + 4) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (r0 + a == p) {
#pragma unroll
          for (int b = 0; b < 8; ++b) row[c0 + b] = v[a][b];
        }
    }
    if (t == 0) rowof[k] = p;
    __syncthreads();
    double d = col[p];
    if (!(d != 0.0) || !isfinite(d)) {
      if (t == 0) *bad = 1;
      d = qnan<double>();
    }
    const double rd = 1.0 / d;
    double rp[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) rp[b] = row[c0 + b] * rd;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = r0 + a;
      const double f = col[i];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int j = c0 + b;
        double x;
        if (i == p) x = (j == k) ? rd : rp[b];
        else x = (j == k) ? -f * rd : fma(-f, rp[b], v[a][b]);
        v[a][b] = x;
      }
    }
  }
  // register (i, j) holds inverse(col_of(i), rowof[j]) where col_of(i) is the
  // column pivoted on row i: invert the pivot map through LDS
  __syncthreads();
  int* colof = rowof + 128;
  for (int k = t; k < n; k += kBT) colof[rowof[k]] = k;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = r0 + a, j = c0 + b;
      if (i < n && j < n) Mx[colof[i] * ld + rowof[j]] = v[a][b];
    }
  __syncthreads();
}

}  // namespace big
}  // namespace lqr
