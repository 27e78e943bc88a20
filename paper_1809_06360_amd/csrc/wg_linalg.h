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

// Global-memory access through a pointer into device memory. Accesses through
// a generic pointer compile to flat_* instructions, which count in lgkmcnt as
// well as vmcnt, so every wait for an LDS access would also wait for all
// global loads and stores in flight; through a global address-space pointer
// they are global_* instructions, counted in vmcnt only.
#define LQR_GLOBAL __attribute__((address_space(1)))
template <typename T>
LQR_DEV LQR_GLOBAL T* gp(T* p) {
  return (LQR_GLOBAL T*)p;
}

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
  const LQR_GLOBAL T* gsrc = gp(src);
  for (int e0 = threadIdx.x; e0 < total; e0 += U * kThreads) {
    T v[U];
    int ii[U], jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ii[u] = i;
      jj[u] = j;
      v[u] = e0 + u * kThreads < total ? gsrc[i * lds + j] : T(0);
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
    dst[i * ldd + j] = gp(src)[j * lds + i];
  }
}

template <typename T>
LQR_DEV void store_block(T* __restrict__ dst, int ldd, const T* src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int i = e / cols, j = e - i * cols;
    gp(dst)[i * ldd + j] = src[i * lds + j];
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
// M1, M2 may live in global memory or LDS; v1, v2 in LDS. Up to 64 rows, four
// lanes share a row (consecutive columns, so a load instruction covers 16 rows
// x 32 bytes) and their partial sums meet by two quad permutations; longer
// matrices take one wave per row with a wave reduction.
// ---------------------------------------------------------------------------
template <int CTRL>
LQR_DEV double quad_xor(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, typename Epi>
LQR_DEV void gemv2(int rows, int c1, const T* M1, int ld1, const T* v1,
                   int c2, const T* M2, int ld2, const T* v2, Epi epi) {
  static_assert(kThreads == 256, "four lanes per row for 64 rows");
  if (rows <= 64) {
    const int i = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int r = i < rows ? i : 0;
    T s0 = T(0), s1 = T(0);
    const T* a1 = M1 + (size_t)r * ld1;
    const T* a2 = M2 + (size_t)r * ld2;
    int l = q;
    for (; l + 4 < c1; l += 8) {
      s0 = fma(a1[l], v1[l], s0);
      s1 = fma(a1[l + 4], v1[l + 4], s1);
    }
    if (l < c1) s0 = fma(a1[l], v1[l], s0);
    for (l = q; l < c2; l += 4) s1 = fma(a2[l], v2[l], s1);
    T s = s0 + s1;
    s += quad_xor<0xB1>(s);  // quad_perm 1,0,3,2
    s += quad_xor<0x4E>(s);  // quad_perm 2,3,0,1
    if (q == 0 && i < rows) epi(i, s);
    return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < rows; i += kWaves) {
    T s = T(0);
    for (int l = lane; l < c1; l += 64) s = fma(M1[i * ld1 + l], v1[l], s);
    for (int l = lane; l < c2; l += 64) s = fma(M2[i * ld2 + l], v2[l], s);
    s = wave_sum(s);
    if (lane == 0) epi(i, s);
  }
}

// Matrix-vector products of at most 64 rows by the 64 lanes of ONE wave
// (`w`; lane i takes row i, four accumulation chains), for blocks in LDS or
// walked along coalesced columns: no cross-lane reduction, so a product costs
// about `cols` dependent loads and multiply-adds, and products handed to
// different waves run side by side.
//   gemv_wave:    y(i) = epi(i, sum_l M[i * ld + l] v[l])   (row-major M)
//   gemv_cm_wave: y(i) = epi(i, sum_l A[l * lda + i] v[l])  (column-major A,
//                 or the transpose of a row-major block)
template <bool ColMajor, typename T, typename Epi>
LQR_DEV void gemv_lanes(int w, int rows, int cols, const T* A, int ld, const T* v, Epi epi) {
  if ((int)(threadIdx.x >> 6) != w) return;
  const int i = threadIdx.x & 63;
  const int r = i < rows ? i : 0;
  T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
  const T* a = ColMajor ? A + r : A + (size_t)r * ld;
  const int st = ColMajor ? ld : 1;
  int l = 0;
  for (; l + 3 < cols; l += 4) {
    s0 = fma(a[l * st], v[l], s0);
    s1 = fma(a[(l + 1) * st], v[l + 1], s1);
    s2 = fma(a[(l + 2) * st], v[l + 2], s2);
    s3 = fma(a[(l + 3) * st], v[l + 3], s3);
  }
  for (; l < cols; ++l) s0 = fma(a[l * st], v[l], s0);
  if (i < rows) epi(i, (s0 + s1) + (s2 + s3));
}

template <typename T, typename Epi>
LQR_DEV void gemv_wave(int w, int rows, int cols, const T* M, int ld, const T* v, Epi epi) {
  gemv_lanes<false>(w, rows, cols, M, ld, v, epi);
}

template <typename T, typename Epi>
LQR_DEV void gemv_cm_wave(int w, int rows, int cols, const T* A, int lda, const T* v, Epi epi) {
  gemv_lanes<true>(w, rows, cols, A, lda, v, epi);
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
          if (i < m) gp(chol)[i * m + lane] = (i == lane) ? sc : (i > lane ? v[i] / sc : 0.0);
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
          if (i < m) gp(chol)[i * m + lane] = (i == lane) ? sc : (i > lane ? v[i] / sc : 0.0);
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
// Inverse of an n x n matrix (n <= 64) by Gauss-Jordan exchange steps with
// row pivoting (wg_invert below). Lane i of every wave holds row i of the
// working table; step k pivots column k on the unused row p of largest
// magnitude and every other row i takes
//   a(i, j) -= a(i, k)/a(p, k) * a(p, j)  (j != k),   a(i, k) /= a(p, k).
// The exchange would also scale the pivot row by -1/a(p, k) (and set its
// pivot entry to 1/a(p, k)); that scale is kept aside per row (sigma, with
// the stored pivot entry -1) and applied once at the end, so a step costs one
// fused multiply-add per element on every lane alike: later steps treat the
// stored row exactly, since the scale cancels from their updates. After n
// steps row i of the table holds row step(i) of the inverse with its columns
// in pivot order: inverse(step(i), p_k) = sigma_i * a(i, k).
// ---------------------------------------------------------------------------
// 1/d by the hardware reciprocal estimate and two Newton steps (quadratic
// convergence from its ~2^-23 relative error: well below 1 ulp of FP64 after
// the second step; exact reciprocals of powers of two). Used where the
// reciprocal is on a serial chain; d is finite and nonzero or NaN.
LQR_DEV double recip(double d) {
  double x = __builtin_amdgcn_rcp(d);
  x = fma(x, fma(-d, x, 1.0), x);
  return fma(x, fma(-d, x, 1.0), x);
}

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

// ---------------------------------------------------------------------------
// The inverse by the four waves of the workgroup: wave w keeps the
// columns j = w, w + 4, ... of the working table (lane i = row i, as above),
// so each step's updates are spread over the four SIMDs; one workgroup
// barrier per step. In step k the wave owning column k + 1 (already updated
// by the steps before k) applies step k to that column first, searches the
// next pivot and publishes its row and the multipliers -a(i, k+1)/a(p, k+1)
// of every row to the double-buffered exchange `xb` (2 * 64 doubles, 2
// doubles and 2 ints of LDS) before updating its other columns, so the
// search overlaps the other waves' updates. Every wave tracks the per-row
// scale, pivot step and pivot rows from what is published. Input element
// (i, j) at A[j * lda + i]; the inverse goes to Ainv with the same
// column-major convention (Ainv may be A: all of A is read before any write).
// A zero or non-finite pivot yields NaN results and returns 1. Called by all
// kThreads threads together; starts and ends with a workgroup barrier.
// ---------------------------------------------------------------------------
struct InvExchange {
  double* c;   // 2 x 64 multipliers
  double* iv;  // 2 reciprocal pivots
  int* p;      // 2 pivot rows
  int* bad;
};

LQR_DEV InvExchange carve_inv_exchange(double* base) {
  InvExchange x;
  x.c = base;
  x.iv = base + 128;
  x.p = reinterpret_cast<int*>(base + 130);
  x.bad = x.p + 2;
  return x;
}
static_assert(kInvExchangeDoubles == 132, "exchange layout");

// Body of wave W (compile-time, so that every column index is a constant).
template <int MAXN, int W>
LQR_DEV int wg_invert_wave(const double* A, int lda, int n, double* Ainv, int ldi, InvExchange x) {
  constexpr int NC = (MAXN + 3) / 4;  // columns per wave
  const int lane = threadIdx.x & 63;
  const bool live = lane < n;
  const int row = live ? lane : 0;
  __syncthreads();  // A is complete
  double a[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int j = 4 * q + W;
    a[q] = A[(j < n ? j : n - 1) * lda + row];
  }
  bool used = !live;
  int step = 0, prow = 0;
  double sigma = 1.0;
  // pivot search on a column held by this wave; publishes the pivot row, its
  // reciprocal and the multipliers of every row into slot s
  auto search = [&](double v, int s) {
    const unsigned hi = (unsigned)(__builtin_bit_cast(unsigned long long, v) >> 32) & 0x7fffffffu;
    const unsigned key = wave_max_u32(used ? 0u : ((hi & ~63u) | (unsigned)(63 - lane)) + 64u);
    const int p = 63 - (int)(key & 63u);
    double piv = readlane(v, p);
    const bool ok = (piv != 0.0) && isfinite(piv);
    piv = ok ? piv : qnan<double>();
    const double inv = recip(piv);
    x.c[s * 64 + lane] = row == p ? 0.0 : -v * inv;
    if (lane == 0) {
      x.iv[s] = inv;
      x.p[s] = p;
      if (!ok) *x.bad = 1;
    }
  };
  if constexpr (W == 0) {
    if (lane == 0) *x.bad = 0;
    search(a[0], 0);
  }
  __syncthreads();
  static_for<0, MAXN>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if (k < n) {
      constexpr int s = k & 1;
      // the owner of column k + 1 applies step k to it first and publishes
      // the next pivot before its other columns
      constexpr int qn = (k + 1) / 4;
      constexpr bool owner = ((k + 1) & 3) == W && qn < NC;
      const double c = x.c[s * 64 + lane];
      const double inv = x.iv[s];
      const int p = __builtin_amdgcn_readfirstlane(x.p[s]);
      const bool isp = row == p;
      if (isp) {
        sigma = -inv;
        used = true;
        step = k;
      }
      if (lane == k) prow = p;
      if constexpr (owner) {
        a[qn] = fma(c, readlane(a[qn], p), a[qn]);
        if (k + 1 < n) search(a[qn], s ^ 1);
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (4 * q + W == k)
          a[q] = isp ? -1.0 : -c;
        else if (!(owner && q == qn))
          a[q] = fma(c, readlane(a[q], p), a[q]);
      }
      __syncthreads();
    }
  });
  // column j = 4q + W of the table is column p_j of the inverse
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int j = 4 * q + W;
    if (j < n) {
      const int col = __builtin_amdgcn_readlane(prow, j);
      if (live) Ainv[col * ldi + step] = sigma * a[q];
    }
  }
  const int bad = *x.bad;
  __syncthreads();
  return bad;
}

template <int MAXN>
LQR_DEV int wg_invert(const double* A, int lda, int n, double* Ainv, int ldi, InvExchange x) {
  static_assert(MAXN <= 64 && kWaves == 4, "one row per lane, four waves");
  switch (threadIdx.x >> 6) {
    case 0: return wg_invert_wave<MAXN, 0>(A, lda, n, Ainv, ldi, x);
    case 1: return wg_invert_wave<MAXN, 1>(A, lda, n, Ainv, ldi, x);
    case 2: return wg_invert_wave<MAXN, 2>(A, lda, n, Ainv, ldi, x);
    default: return wg_invert_wave<MAXN, 3>(A, lda, n, Ainv, ldi, x);
  }
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

// One operand stream of a pair of tiles (tile 1 only if `two`): per lane the
// fragment addresses are formed once (rows and columns clamped into the
// operands; out-of-range rows and columns only reach discarded outputs) and
// walked by constant strides; the k range runs in chunks of 16 (four MFMAs per
// tile) with the next chunk's fragments loaded before the current chunk's
// MFMAs, and a last partial chunk whose out-of-range k are zeroed. NEG
// subtracts the product.
template <bool TA, bool TB, bool NEG>
LQR_DEV void mfma_pair(f64x4& acc0, f64x4& acc1, bool two, const double* A, int lda, const double* B,
                       int ldb, int M, int N, int K, int i0, int j0, int i1, int j1, int li, int lk) {
  const int ra0 = min(i0 + li, M - 1), cb0 = min(j0 + li, N - 1);
  const int ra1 = min(i1 + li, M - 1), cb1 = min(j1 + li, N - 1);
  const int sa = TA ? 4 * lda : 4, sb = TB ? 4 : 4 * ldb;  // one k-step of 4
  const double* pa0 = TA ? A + lk * lda + ra0 : A + ra0 * lda + lk;
  const double* pa1 = TA ? A + lk * lda + ra1 : A + ra1 * lda + lk;
  const double* pb0 = TB ? B + cb0 * ldb + lk : B + lk * ldb + cb0;
  const double* pb1 = TB ? B + cb1 * ldb + lk : B + lk * ldb + cb1;
  const int full = K >> 4;
  double a0[4], b0[4], a1[4], b1[4];
  auto load = [&](int c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a0[s] = pa0[(4 * c + s) * sa];
      b0[s] = pb0[(4 * c + s) * sb];
    }
    if (two) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a1[s] = pa1[(4 * c + s) * sa];
        b1[s] = pb1[(4 * c + s) * sb];
      }
    }
  };
  if (full > 0) load(0);
  for (int c = 0; c < full; ++c) {
    double x0[4], y0[4], x1[4], y1[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      x0[s] = a0[s];
      y0[s] = b0[s];
      x1[s] = a1[s];
      y1[s] = b1[s];
    }
    if (c + 1 < full) load(c + 1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -x0[s] : x0[s], y0[s], acc0, 0, 0, 0);
      if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -x1[s] : x1[s], y1[s], acc1, 0, 0, 0);
    }
  }
  const int k0 = full << 4;
  if (k0 < K) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * s + lk;
      const bool kin = k < K;
      const int st = ((kin ? k : K - 1) - lk) >> 2;  // clamped k-step of this lane's row
      const double xa0 = kin ? pa0[st * sa] : 0.0, xb0 = kin ? pb0[st * sb] : 0.0;
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -xa0 : xa0, xb0, acc0, 0, 0, 0);
      if (two) {
        const double xa1 = kin ? pa1[st * sa] : 0.0, xb1 = kin ? pb1[st * sb] : 0.0;
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -xa1 : xa1, xb1, acc1, 0, 0, 0);
      }
    }
  }
}

template <bool TA1, bool TB1, bool TA2, bool TB2, typename Epi, typename Skip = NoSkip>
LQR_DEV void mgemm_sub(int M, int N,
                       int K1, const double* A1, int lda1, const double* B1, int ldb1,
                       int K2, const double* A2, int lda2, const double* B2, int ldb2,
                       Epi epi, Skip skip = Skip()) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tn = (N + 15) >> 4;
  const int tiles = ((M + 15) >> 4) * tn;
  for (int t0 = wave; t0 < tiles; t0 += 2 * kWaves) {
    const int t1 = t0 + kWaves;
    int ia = (t0 / tn) << 4, ja = (t0 % tn) << 4;
    int ib = t1 < tiles ? (t1 / tn) << 4 : ia, jb = t1 < tiles ? (t1 % tn) << 4 : ja;
    bool runa = !skip(ia, ja, 16, 16);
    bool runb = t1 < tiles && !skip(ib, jb, 16, 16);
    if (!runa && !runb) continue;
    if (!runa) {  // only the second tile: compute it in the first slot
      ia = ib;
      ja = jb;
      runa = true;
      runb = false;
    }
    f64x4 acca = {0.0, 0.0, 0.0, 0.0}, accb = {0.0, 0.0, 0.0, 0.0};
    if (K1 > 0) mfma_pair<TA1, TB1, false>(acca, accb, runb, A1, lda1, B1, ldb1, M, N, K1, ia, ja, ib, jb, li, lk);
    if (K2 > 0) mfma_pair<TA2, TB2, true>(acca, accb, runb, A2, lda2, B2, ldb2, M, N, K2, ia, ja, ib, jb, li, lk);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = lk + 4 * r;
      if (ia + i < M && ja + li < N) epi(ia + i, ja + li, acca[r]);
      if (runb && ib + i < M && jb + li < N) epi(ib + i, jb + li, accb[r]);
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
