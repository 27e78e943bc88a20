// Workgroup-level dense linear algebra on LDS-resident blocks, for gfx950.
//
// Every routine here is called by all threads of a 256-thread workgroup
// (4 wave64s) with identical arguments; operands and results live in LDS
// unless stated otherwise. Routines do not synchronise at their end: callers
// place __syncthreads() between a producer and its consumers. All index
// arithmetic is 32-bit; matrices are row-major with an explicit leading
// dimension.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lqr_layout.h"

#define LQR_DEV __device__ __forceinline__

namespace lqr {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T>
LQR_DEV T qnan() { return __builtin_nan(""); }

// Element (i, j) of op(X) where op is identity or transpose.
template <bool Trans, typename T>
LQR_DEV T el(const T* p, int ld, int i, int j) {
  return Trans ? p[j * ld + i] : p[i * ld + j];
}

// ---------------------------------------------------------------------------
// Register-tiled product with an optional subtracted second product:
//   v(i, j) = sum_k op(A1)(i,k) op(B1)(k,j)  -  sum_k op(A2)(i,k) op(B2)(k,j)
// for 0 <= i < M, 0 <= j < N, handed to epi(i, j, v). Each thread owns RMxRN
// output tiles (tile index strided by the block size); operand indices are
// clamped so every load stays inside the operands, and only in-range outputs
// reach the epilogue. `skip(i0, j0)` may drop whole tiles (e.g. the strictly
// upper tiles of a symmetric result).
// ---------------------------------------------------------------------------
struct NoSkip {
  LQR_DEV bool operator()(int, int, int, int) const { return false; }
};

// Drop tiles (rows i0.., columns j0.., extent tm x tn) lying strictly above the
// diagonal of the leading `ns` x `ns` block. A tile is dropped only if all its
// columns lie inside that block, so tiles that also hold columns >= ns are
// always computed.
struct SkipUpper {
  int ns;
  LQR_DEV bool operator()(int i0, int j0, int tm, int tn) const {
    return j0 + tn <= ns && j0 > i0 + tm - 1;
  }
};

// Same, for a symmetric block stored in output columns [coff, coff + ns).
struct SkipUpperShift {
  int ns, coff;
  LQR_DEV bool operator()(int i0, int j0, int tm, int tn) const {
    return j0 >= coff && j0 + tn <= coff + ns && j0 - coff > i0 + tm - 1;
  }
};

template <int RM, int RN, bool TA1, bool TB1, bool TA2, bool TB2, typename T, typename Epi,
          typename Skip = NoSkip>
LQR_DEV void gemm_sub(int M, int N,
                      int K1, const T* A1, int lda1, const T* B1, int ldb1,
                      int K2, const T* A2, int lda2, const T* B2, int ldb2,
                      Epi epi, Skip skip = Skip()) {
  const int tn = (N + RN - 1) / RN;
  const int tiles = ((M + RM - 1) / RM) * tn;
  for (int tile = threadIdx.x; tile < tiles; tile += kThreads) {
    const int i0 = (tile / tn) * RM, j0 = (tile % tn) * RN;
    if (skip(i0, j0, RM, RN)) continue;
    int ii[RM], jj[RN];
#pragma unroll
    for (int r = 0; r < RM; ++r) ii[r] = min(i0 + r, M - 1);
#pragma unroll
    for (int s = 0; s < RN; ++s) jj[s] = min(j0 + s, N - 1);
    T acc[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int s = 0; s < RN; ++s) acc[r][s] = T(0);
    for (int k = 0; k < K1; ++k) {
      T a[RM], b[RN];
#pragma unroll
      for (int r = 0; r < RM; ++r) a[r] = el<TA1>(A1, lda1, ii[r], k);
#pragma unroll
      for (int s = 0; s < RN; ++s) b[s] = el<TB1>(B1, ldb1, k, jj[s]);
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int s = 0; s < RN; ++s) acc[r][s] = fma(a[r], b[s], acc[r][s]);
    }
    for (int k = 0; k < K2; ++k) {
      T a[RM], b[RN];
#pragma unroll
      for (int r = 0; r < RM; ++r) a[r] = el<TA2>(A2, lda2, ii[r], k);
#pragma unroll
      for (int s = 0; s < RN; ++s) b[s] = el<TB2>(B2, ldb2, k, jj[s]);
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int s = 0; s < RN; ++s) acc[r][s] = fma(-a[r], b[s], acc[r][s]);
    }
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int s = 0; s < RN; ++s)
        if (i0 + r < M && j0 + s < N) epi(i0 + r, j0 + s, acc[r][s]);
  }
}

template <int RM, int RN, bool TA, bool TB, typename T, typename Epi, typename Skip = NoSkip>
LQR_DEV void gemm(int M, int N, int K, const T* A, int lda, const T* B, int ldb, Epi epi,
                  Skip skip = Skip()) {
  gemm_sub<RM, RN, TA, TB, false, false>(M, N, K, A, lda, B, ldb, 0, A, lda, B, ldb, epi, skip);
}

// ---------------------------------------------------------------------------
// Copies between global memory and LDS (row-major, rows x cols).
// ---------------------------------------------------------------------------
// load_block issues up to U loads per thread before it stores any of them, so
// a block costs about one memory round trip per U * kThreads elements. A
// thread's elements are kThreads apart; (i, j) advance without divisions.
template <typename T>
LQR_DEV void load_block(T* dst, int ldd, const T* __restrict__ src, int lds, int rows, int cols) {
  constexpr int U = 8;
  const int total = rows * cols;
  const int di = kThreads / cols, dj = kThreads - di * cols;
  int i = threadIdx.x / cols, j = threadIdx.x - i * cols;
  for (int e0 = threadIdx.x; e0 < total; e0 += U * kThreads) {
    T v[U];
    int ii[U], jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ii[u] = i;
      jj[u] = j;
      v[u] = e0 + u * kThreads < total ? src[i * lds + j] : T(0);
      i += di;
      j += dj;
      if (j >= cols) {
        j -= cols;
        ++i;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * kThreads < total) dst[ii[u] * ldd + jj[u]] = v[u];
  }
}

// dst (rows x cols) = transpose of src (cols x rows, leading dimension lds).
template <typename T>
LQR_DEV void load_block_t(T* dst, int ldd, const T* __restrict__ src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int j = e / rows, i = e - j * rows;   // consecutive threads walk a source row
    dst[i * ldd + j] = src[j * lds + i];
  }
}

template <typename T>
LQR_DEV void store_block(T* __restrict__ dst, int ldd, const T* src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

template <typename T>
LQR_DEV void fill_block(T* dst, int ldd, int rows, int cols, T v, T diag) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = (i == j) ? diag : v;
  }
}

// ---------------------------------------------------------------------------
// Wave reductions.
// ---------------------------------------------------------------------------
template <typename T>
LQR_DEV T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// y(i) = epi(i, sum_l M1[i][l] v1[l] + sum_l M2[i][l] v2[l]) for i < rows.
// M1, M2 may live in global memory or LDS; v1, v2 in LDS. One wave per row,
// lanes stride the columns (coalesced row reads), wave-reduced.
// ---------------------------------------------------------------------------
template <typename T, typename Epi>
LQR_DEV void gemv2(int rows, int c1, const T* M1, int ld1, const T* v1,
                   int c2, const T* M2, int ld2, const T* v2, Epi epi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < rows; i += kWaves) {
    T s = T(0);
    for (int l = lane; l < c1; l += 64) s = fma(M1[i * ld1 + l], v1[l], s);
    for (int l = lane; l < c2; l += 64) s = fma(M2[i * ld2 + l], v2[l], s);
    s = wave_sum(s);
    if (lane == 0) epi(i, s);
  }
}

// y(i) = epi(i, sum_l A[l * lda + i] v[l]) for i < rows <= kThreads: a
// column-major A (or the transpose of a row-major block); thread i walks row i
// with two accumulation chains.
template <typename T, typename Epi>
LQR_DEV void gemv_cm(int rows, int cols, const T* A, int lda, const T* v, Epi epi) {
  const int i = threadIdx.x;
  if (i < rows) {
    T s0 = T(0), s1 = T(0);
    int l = 0;
    for (; l + 1 < cols; l += 2) {
      s0 = fma(A[l * lda + i], v[l], s0);
      s1 = fma(A[(l + 1) * lda + i], v[l + 1], s1);
    }
    if (l < cols) s0 = fma(A[l * lda + i], v[l], s0);
    epi(i, s0 + s1);
  }
}

// ---------------------------------------------------------------------------
// Cross-lane helpers.
// ---------------------------------------------------------------------------
// Value of v in lane `lane` (uniform lane index) broadcast to the wave.
LQR_DEV double readlane(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// Register capacity for an m x m factor: 8, 16, 32 or 64 (m <= 64). Blocks
// handed to the factorization routines use this as their leading dimension,
// so every unrolled access has a compile-time offset.
// ---------------------------------------------------------------------------
LQR_HD int pad_m(int m) { return pad_rows(m); }
// Leading dimension used with capacity MAXM: one more than MAXM, so that a
// column walk by 16 lanes hits distinct LDS banks.
LQR_HD int pad_ld(int m) { return pad_rows(m) + 1; }

// ---------------------------------------------------------------------------
// Square-root-free Cholesky (L D L') of the m x m input Hessian H and forward
// elimination of a set of right-hand sides. G is column-major in LDS with
// leading dimension ldg: columns [0, m) hold H, [m, m + nr) the right-hand
// sides; if `ident`, m more right-hand sides are the identity (not stored).
//  1. Wave 0 factors H with lane k holding column k in registers. In round k
//     every lane reads the pivot d_k and column k from lane k (readlane) and
//     lane c > k updates its rows i > k by -H(i, k) H(k, c) / d_k: the trailing
//     block stays symmetric, so lane c's own row-k entry is H(k, c). No
//     barrier inside the factorization. Lane k then stores the multipliers
//     H(i, k)/d_k (i > k) over H's column k in G and 1/sqrt(d_k) to buf.
//  2. Every right-hand side (one thread per column) runs the unit-lower
//     forward substitution with those multipliers and scales row i by
//     1/sqrt(d_i).
// When MAXM <= 32 and the right-hand sides fit in the waves' spare lanes
// (kWaves (64 - m) of them), every wave instead factors H redundantly in
// lanes [0, m) and carries its share of the right-hand sides in lanes
// [m, 64): a right-hand side y takes the same round-k update as H's columns,
// y_i -= H(i, k) (y_k / d_k), so step 2 and its barriers disappear; the
// waves compute identical factors.
// The loops are unrolled for m <= MAXM so every register index is fixed.
//
// On return (ends with a barrier):
//   Z = L^{-1} X  for every right-hand side X (L = L_unit D^{1/2} the
//     Cholesky factor), written to G's columns [m, m + nr);
//   if ident: L^{-1} written to zi (column q of L^{-1} at zi + q * ldzi);
//   if chol != nullptr: L written row-major to chol (m x m, zeros above);
//   G's columns [0, m) hold the multipliers (unless zi overwrote them).
// A pivot that is not positive or not finite is replaced by NaN (which then
// propagates into every dependent result) and *bad is set: to 1 if the first
// such pivot was finite (H not positive definite), to 2 if it was not finite.
// buf: MAXM doubles of LDS. Requires m <= 64, m + nr + (ident ? m : 0) <= 256
// and a barrier between G's producer and this call.
// ---------------------------------------------------------------------------
template <int MAXM>
LQR_DEV void ldl_columns(double* G, int ldg, int m, int nr, bool ident, double* zi, int ldzi,
                         double* chol, double* buf, int* bad) {
  const int c = threadIdx.x;
  const int lane = c & 63;
  const int wave = __builtin_amdgcn_readfirstlane(c >> 6);
  if constexpr (MAXM <= 32) {
    const int nrhs = nr + (ident ? m : 0), per = 64 - m;
    if (kWaves * per >= nrhs) {
      const bool isH = lane < m;
      const int r = wave * per + lane - m;  // right-hand side of this lane
      const bool isR = !isH && r < nrhs;
      const bool fromG = isR && r < nr;
      const int q = r - nr;                 // identity column
      const double* src = G + (isH ? lane : fromG ? m + r : 0) * ldg;
      double v[MAXM];
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        v[i] = i < m ? ((isH || fromG) ? src[i] : ((isR && i == q) ? 1.0 : 0.0)) : 0.0;
      __syncthreads();  // every wave has read H before any result overwrites it
      int badf = 0;
#pragma unroll
      for (int k = 0; k < MAXM; ++k) {
        if (k < m) {
          double dk = readlane(v[k], k);
          if (!(dk > 0.0) || !isfinite(dk)) {
            if (!badf) badf = isfinite(dk) ? 1 : 2;
            dk = qnan<double>();
          }
          const double s = (isR || lane > k) ? v[k] / dk : 0.0;
#pragma unroll
          for (int i = k + 1; i < MAXM; ++i) v[i] = fma(-readlane(v[i], k), s, v[i]);
        }
      }
      // lane c < m: pivot d_c, scale 1/sqrt(d_c); right-hand sides: row i times 1/sqrt(d_i)
      double dc = v[0];
#pragma unroll
      for (int i = 1; i < MAXM; ++i)
        if (i == lane) dc = v[i];
      if (!(dc > 0.0) || !isfinite(dc)) dc = qnan<double>();
      const double sc = sqrt(dc), rs = 1.0 / sc;
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i < m) {
          const double ri = readlane(rs, i);
          if (isR) v[i] *= ri;
        }
      if (wave == 0 && isH && chol) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
          if (i < m) chol[i * m + lane] = (i == lane) ? sc : (i > lane ? v[i] / sc : 0.0);
      }
      if (isR) {
        double* dst = fromG ? G + (m + r) * ldg : zi + q * ldzi;
#pragma unroll
        for (int i = 0; i < MAXM; ++i) dst[i] = v[i];
      }
      if (badf && wave == 0 && lane == 0) *bad = badf;
      __syncthreads();
      return;
    }
  }
  if (wave == 0) {
    // rows m..MAXM-1 and lanes m..63 are zero padding: they stay zero
    double v[MAXM];
    const bool isH = lane < m;
    const double* src = G + (isH ? lane : 0) * ldg;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) v[i] = (isH && i < m) ? src[i] : 0.0;
    int badf = 0;
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
      if (k < m) {
        double dk = readlane(v[k], k);
        if (!(dk > 0.0) || !isfinite(dk)) {
          if (!badf) badf = isfinite(dk) ? 1 : 2;
          dk = qnan<double>();
        }
        const double s = lane > k ? v[k] / dk : 0.0;
#pragma unroll
        for (int i = k + 1; i < MAXM; ++i) v[i] = fma(-readlane(v[i], k), s, v[i]);
      }
    }
    if (isH) {
      double dc = v[0];
#pragma unroll
      for (int i = 1; i < MAXM; ++i)
        if (i == lane) dc = v[i];
      if (!(dc > 0.0) || !isfinite(dc)) dc = qnan<double>();
      const double inv = 1.0 / dc, sc = sqrt(dc);
      double* col = G + lane * ldg;
#pragma unroll
      for (int i = 0; i < MAXM; ++i)
        if (i > lane) col[i] = v[i] * inv;
      buf[lane] = 1.0 / sc;
      if (chol) {
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
          if (i < m) chol[i * m + lane] = (i == lane) ? sc : (i > lane ? v[i] / sc : 0.0);
      }
    }
    if (badf && lane == 0) *bad = badf;
  }
  __syncthreads();
  const int nvc = m + nr + (ident ? m : 0);
  const bool own = c >= m && c < nvc;
  const bool fromG = c < m + nr;
  const int q = c - m - nr;
  double v[MAXM];
  if (own) {
    const double* src = G + (fromG ? c : 0) * ldg;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) v[i] = i < m ? (fromG ? src[i] : (i == q ? 1.0 : 0.0)) : 0.0;
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
      if (k < m) {
        const double rk = v[k];
        const double* mk = G + k * ldg;
#pragma unroll
        for (int i = k + 1; i < MAXM; ++i) v[i] = fma(-mk[i], rk, v[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
      if (i < m) v[i] *= buf[i];
  }
  __syncthreads();
  if (own) {
    double* dst = fromG ? G + c * ldg : zi + q * ldzi;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) dst[i] = v[i];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Inverse of an n x n matrix (n <= MAXN <= 64) by ONE wave, with no workgroup
// barrier: Gauss-Jordan exchange steps with row pivoting. Lane i keeps row i
// of the working table in registers; step k pivots column k on the unused row
// p of largest magnitude (a max-reduction over lanes), lane p hands its row to
// the wave through `rowbuf` (LDS, ordered by the wave's own in-order LDS
// queue) and every other row i takes
//   a(i, j) -= a(i, k)/a(p, k) * a(p, j)  (j != k),   a(i, k) /= a(p, k).
// The exchange would also scale the pivot row by -1/a(p, k); that scale is
// kept aside per lane (sigma) and applied once at the end, so a step costs
// one fused multiply-add per element on every lane alike (later steps treat
// the stored row exactly, since the scale cancels from their updates). After
// n steps lane i holds row step(i) of the inverse with its columns in pivot
// order: inverse(step(i), p_k) = sigma_i * a(i, k).
// Input element (i, j) at A[j * lda + i]; the inverse goes to Ainv with the
// same column-major convention (Ainv may be A: all of A is read before any
// write). A zero or non-finite pivot yields NaN results and returns 1.
// Called by the 64 lanes of one wave together; the caller orders the producer
// of A and the consumers of Ainv with workgroup barriers.
// ---------------------------------------------------------------------------
// Largest unsigned value over the wave (all 64 lanes active).
LQR_DEV unsigned wave_max_u32(unsigned v) {
  unsigned o;
  o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v = v > o ? v : o;
  o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  v = v > o ? v : o;
  o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v = v > o ? v : o;
  o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  v = v > o ? v : o;
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  const unsigned s0 = r0 > r1 ? r0 : r1, s1 = r2 > r3 ? r2 : r3;
  return s0 > s1 ? s0 : s1;
}

// Compile-time loop: f(Int<I>{}) for I in [B, E), so that register arrays
// indexed by the loop variable stay in registers however long the body is.
template <int V>
struct Int {
  static constexpr int value = V;
};
template <int B, int E, typename F>
LQR_DEV void static_for(F&& f) {
  if constexpr (B < E) {
    f(Int<B>{});
    static_for<B + 1, E>(f);
  }
}

template <int MAXN>
LQR_DEV int wave_invert(const double* A, int lda, int n, double* Ainv, int ldi, double* rowbuf) {
  static_assert(MAXN <= 64, "one row per lane");
  const int lane = threadIdx.x & 63;
  const bool live = lane < n;
  // Rows past n (lanes that never pivot) and columns past n are padding: they
  // load clamped copies and are never read back into the first n columns.
  const int row = live ? lane : 0;
  double a[MAXN];
#pragma unroll
  for (int j = 0; j < MAXN; ++j) a[j] = A[(j < n ? j : n - 1) * lda + row];
  bool used = !live;
  int step = 0, prow = 0, bad = 0;
  double sigma = 1.0;
  static_for<0, MAXN>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if (k < n) {
      // pivot: largest |a(i, k)| over unused rows. Key = high word of |a|
      // (exponent and leading mantissa bits) with its low 6 bits replaced by
      // 63 - lane (ties go to the lowest row), offset so that any unused row
      // outranks the used ones; NaN and infinity rank first.
      const unsigned hi = (unsigned)(__builtin_bit_cast(unsigned long long, a[k]) >> 32) & 0x7fffffffu;
      const unsigned key = wave_max_u32(used ? 0u : ((hi & ~63u) | (unsigned)(63 - lane)) + 64u);
      const int p = 63 - (int)(key & 63u);
      double piv = readlane(a[k], p);
      if (!(piv != 0.0) || !isfinite(piv)) {
        bad = 1;
        piv = qnan<double>();
      }
      const double inv = 1.0 / piv;
      const bool isp = lane == p;
      // the previous step's reads of rowbuf precede this store, and the store
      // precedes this step's reads (LDS is in order within a wave; the fences
      // keep the compiler from moving the accesses across lanes' boundaries)
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (isp) {
#pragma unroll
        for (int j = 0; j < MAXN; ++j) rowbuf[j] = a[j];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // the whole pivot row is requested before the first use
      double r[MAXN];
#pragma unroll
      for (int j = 0; j < MAXN; ++j) r[j] = rowbuf[j];
      __builtin_amdgcn_sched_barrier(0);
      const double g = a[k] * inv;
      const double c = isp ? 0.0 : -g;
#pragma unroll
      for (int j = 0; j < MAXN; ++j)
        if (j != k) a[j] = fma(c, r[j], a[j]);
      a[k] = isp ? -1.0 : g;
      if (isp) {
        sigma = -inv;
        used = true;
        step = k;
      }
      if (lane == k) prow = p;
    }
  });
#pragma unroll
  for (int k = 0; k < MAXN; ++k) {
    if (k < n) {
      const int col = __builtin_amdgcn_readlane(prow, k);
      if (live) Ainv[col * ldi + step] = sigma * a[k];
    }
  }
  return bad;
}

// ---------------------------------------------------------------------------
// FP64 matrix-core product on 16x16 output tiles (v_mfma_f64_16x16x4f64):
//   v(i, j) = sum_k op(A1)(i,k) op(B1)(k,j) - sum_k op(A2)(i,k) op(B2)(k,j)
// for 0 <= i < M, 0 <= j < N, handed to epi(i, j, v). Operand layout of the
// instruction: lane l supplies A(i = l%16, k = l/16) and B(k = l/16, j = l%16);
// result register r of lane l is D(i = l/16 + 4r, j = l%16). Each wave takes
// every 4th tile and runs two tiles at a time for two independent
// accumulation chains; out-of-range operand elements load as zero.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((vector_size(32)));

// One operand stream of a tile: kc consecutive k-steps (4 k each) of A and B
// fragments loaded up front (independent LDS reads), then kc MFMAs.
template <bool TA, bool TB, int KC>
LQR_DEV void mfma_chunk(f64x4& acc, const double* A, int lda, const double* B, int ldb, int M, int N,
                        int K, int i, int j, int k0, int lk, double sgn) {
  double a[KC], b[KC];
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    const int k = k0 + 4 * s + lk;
    const bool kin = k < K;
    const int kk = kin ? k : K - 1;
    a[s] = (kin && i < M) ? sgn * el<TA>(A, lda, i < M ? i : M - 1, kk) : 0.0;
    b[s] = (kin && j < N) ? el<TB>(B, ldb, kk, j < N ? j : N - 1) : 0.0;
  }
#pragma unroll
  for (int s = 0; s < KC; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
}

template <bool TA1, bool TB1, bool TA2, bool TB2, typename Epi, typename Skip = NoSkip>
LQR_DEV void mgemm_sub(int M, int N,
                       int K1, const double* A1, int lda1, const double* B1, int ldb1,
                       int K2, const double* A2, int lda2, const double* B2, int ldb2,
                       Epi epi, Skip skip = Skip()) {
  constexpr int KC = 4;  // k-steps per preloaded chunk (16 k)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tn = (N + 15) >> 4;
  const int tiles = ((M + 15) >> 4) * tn;
  for (int t0 = wave; t0 < tiles; t0 += 2 * kWaves) {
    const int t1 = t0 + kWaves;
    const bool has1 = t1 < tiles;
    const int i0a = (t0 / tn) << 4, j0a = (t0 % tn) << 4;
    const int i0b = has1 ? (t1 / tn) << 4 : i0a, j0b = has1 ? (t1 % tn) << 4 : j0a;
    const bool runa = !skip(i0a, j0a, 16, 16), runb = has1 && !skip(i0b, j0b, 16, 16);
    if (!runa && !runb) continue;
    f64x4 acca = {0.0, 0.0, 0.0, 0.0}, accb = {0.0, 0.0, 0.0, 0.0};
    const int ia = i0a + li, ja = j0a + li, ib = i0b + li, jb = j0b + li;
    for (int k0 = 0; k0 < K1; k0 += 4 * KC) {
      mfma_chunk<TA1, TB1, KC>(acca, A1, lda1, B1, ldb1, M, N, K1, ia, ja, k0, lk, 1.0);
      if (has1) mfma_chunk<TA1, TB1, KC>(accb, A1, lda1, B1, ldb1, M, N, K1, ib, jb, k0, lk, 1.0);
    }
    for (int k0 = 0; k0 < K2; k0 += 4 * KC) {
      mfma_chunk<TA2, TB2, KC>(acca, A2, lda2, B2, ldb2, M, N, K2, ia, ja, k0, lk, -1.0);
      if (has1) mfma_chunk<TA2, TB2, KC>(accb, A2, lda2, B2, ldb2, M, N, K2, ib, jb, k0, lk, -1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = lk + 4 * r;
      if (runa && i0a + i < M && j0a + li < N) epi(i0a + i, j0a + li, acca[r]);
      if (runb && i0b + i < M && j0b + li < N) epi(i0b + i, j0b + li, accb[r]);
    }
  }
}

template <bool TA, bool TB, typename Epi, typename Skip = NoSkip>
LQR_DEV void mgemm(int M, int N, int K, const double* A, int lda, const double* B, int ldb, Epi epi,
                   Skip skip = Skip()) {
  mgemm_sub<TA, TB, false, false>(M, N, K, A, lda, B, ldb, 0, A, lda, B, ldb, epi, skip);
}

// ---------------------------------------------------------------------------
// FP32 matrix-core product for the mixed-precision mode
// (v_mfma_f32_16x16x4f32): operands are read from their FP64 storage and
// rounded to float, products accumulate in float, and epi receives the float
// sum widened to double. Operand layout as for the FP64 instruction; result
// register r of lane l is D(i = 4 (l/16) + r, j = l%16).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((vector_size(16)));

template <bool TA, bool TB, int KC>
LQR_DEV void mfma32_chunk(f32x4& acc, const double* A, int lda, const double* B, int ldb, int M, int N,
                          int K, int i, int j, int k0, int lk, float sgn) {
  float a[KC], b[KC];
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    const int k = k0 + 4 * s + lk;
    const bool kin = k < K;
    const int kk = kin ? k : K - 1;
    a[s] = (kin && i < M) ? sgn * (float)el<TA>(A, lda, i < M ? i : M - 1, kk) : 0.0f;
    b[s] = (kin && j < N) ? (float)el<TB>(B, ldb, kk, j < N ? j : N - 1) : 0.0f;
  }
#pragma unroll
  for (int s = 0; s < KC; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
}

template <bool TA1, bool TB1, bool TA2, bool TB2, typename Epi, typename Skip = NoSkip>
LQR_DEV void m32gemm_sub(int M, int N,
                         int K1, const double* A1, int lda1, const double* B1, int ldb1,
                         int K2, const double* A2, int lda2, const double* B2, int ldb2,
                         Epi epi, Skip skip = Skip()) {
  constexpr int KC = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tn = (N + 15) >> 4;
  const int tiles = ((M + 15) >> 4) * tn;
  for (int t0 = wave; t0 < tiles; t0 += 2 * kWaves) {
    const int t1 = t0 + kWaves;
    const bool has1 = t1 < tiles;
    const int i0a = (t0 / tn) << 4, j0a = (t0 % tn) << 4;
    const int i0b = has1 ? (t1 / tn) << 4 : i0a, j0b = has1 ? (t1 % tn) << 4 : j0a;
    const bool runa = !skip(i0a, j0a, 16, 16), runb = has1 && !skip(i0b, j0b, 16, 16);
    if (!runa && !runb) continue;
    f32x4 acca = {0.0f, 0.0f, 0.0f, 0.0f}, accb = {0.0f, 0.0f, 0.0f, 0.0f};
    const int ia = i0a + li, ja = j0a + li, ib = i0b + li, jb = j0b + li;
    for (int k0 = 0; k0 < K1; k0 += 4 * KC) {
      mfma32_chunk<TA1, TB1, KC>(acca, A1, lda1, B1, ldb1, M, N, K1, ia, ja, k0, lk, 1.0f);
      if (has1) mfma32_chunk<TA1, TB1, KC>(accb, A1, lda1, B1, ldb1, M, N, K1, ib, jb, k0, lk, 1.0f);
    }
    for (int k0 = 0; k0 < K2; k0 += 4 * KC) {
      mfma32_chunk<TA2, TB2, KC>(acca, A2, lda2, B2, ldb2, M, N, K2, ia, ja, k0, lk, -1.0f);
      if (has1) mfma32_chunk<TA2, TB2, KC>(accb, A2, lda2, B2, ldb2, M, N, K2, ib, jb, k0, lk, -1.0f);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * lk + r;
      if (runa && i0a + i < M && j0a + li < N) epi(i0a + i, j0a + li, (double)acca[r]);
      if (runb && i0b + i < M && j0b + li < N) epi(i0b + i, j0b + li, (double)accb[r]);
    }
  }
}

// Product engines. E = 0: FP64 on the vector ALUs with 4x4 register tiles
// (problems with fewer than 32 states); E = 1: FP64 matrix cores; E = 2: FP32
// matrix cores with FP32 accumulation (mixed-precision mode).
constexpr int kEngValu = 0, kEngMfma64 = 1, kEngMfma32 = 2;

// The FP64 engine that stands in for E where the product must stay in FP64
// (Cholesky solves, gains, the linking solve).
LQR_HD constexpr int fp64_engine(int E) { return E == kEngMfma32 ? kEngMfma64 : E; }

template <int E, bool TA1, bool TB1, bool TA2, bool TB2, typename Epi, typename Skip = NoSkip>
LQR_DEV void pgemm_sub(int M, int N,
                       int K1, const double* A1, int lda1, const double* B1, int ldb1,
                       int K2, const double* A2, int lda2, const double* B2, int ldb2,
                       Epi epi, Skip skip = Skip()) {
  if constexpr (E == kEngMfma32)
    m32gemm_sub<TA1, TB1, TA2, TB2>(M, N, K1, A1, lda1, B1, ldb1, K2, A2, lda2, B2, ldb2, epi, skip);
  else if constexpr (E == kEngMfma64)
    mgemm_sub<TA1, TB1, TA2, TB2>(M, N, K1, A1, lda1, B1, ldb1, K2, A2, lda2, B2, ldb2, epi, skip);
  else
    gemm_sub<4, 4, TA1, TB1, TA2, TB2>(M, N, K1, A1, lda1, B1, ldb1, K2, A2, lda2, B2, ldb2, epi, skip);
}

}  // namespace lqr
