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
  LQR_DEV bool operator()(int, int) const { return false; }
};

// Drop tiles lying strictly above the diagonal of the leading `ns` x `ns`
// block. A tile is dropped only if all its columns lie inside that block, so
// tiles that also hold columns >= ns are always computed.
template <int RM, int RN>
struct SkipUpper {
  int ns;
  LQR_DEV bool operator()(int i0, int j0) const { return j0 + RN <= ns && j0 > i0 + RM - 1; }
};

// Same, for a symmetric block stored in output columns [coff, coff + ns).
template <int RM, int RN>
struct SkipUpperShift {
  int ns, coff;
  LQR_DEV bool operator()(int i0, int j0) const {
    return j0 >= coff && j0 + RN <= coff + ns && j0 - coff > i0 + RM - 1;
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
    if (skip(i0, j0)) continue;
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
template <typename T>
LQR_DEV void load_block(T* dst, int ldd, const T* __restrict__ src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = src[i * lds + j];
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

// ---------------------------------------------------------------------------
// Square-root-free Cholesky (L D L') of the symmetric block
// H = G[0:m, h0:h0+m], carried out as forward elimination on every column of
// G (m rounds, one barrier each). Only H's upper triangle is read. On return
// d[k] (LDS) holds the k-th pivot; row k of G holds (D L')[k, :] in the H
// block (columns h0+k .. h0+m-1) and (L^{-1}_unit X)[k, :] in every column
// outside the H block. A pivot that is not positive or not finite is
// replaced by NaN (which then propagates into every dependent result) and
// the stage is reported through *bad (LDS int, set to 1).
// Requires a barrier between G's producer and this call.
// ---------------------------------------------------------------------------
template <typename T>
LQR_DEV void ldl_forward(T* G, int ldg, int m, int ncols, int h0, T* d, int* bad) {
  for (int k = 0; k < m; ++k) {
    T dk = G[k * ldg + h0 + k];
    if (!(dk > T(0)) || !isfinite(dk)) {
      dk = qnan<T>();
      if (threadIdx.x == 0) *bad = 1;
    }
    if (threadIdx.x == 0) d[k] = dk;
    const T inv = T(1) / dk;
    const int rows = m - k - 1;
    if (rows > 0) {
      // thread -> (column j, row phase); `tpc` threads share a column
      const int tpc = max(1, min(rows, kThreads / ncols));
      for (int idx = threadIdx.x; idx < ncols * tpc; idx += kThreads) {
        const int j = idx % ncols, ph = idx / ncols;
        const int jh = j - h0;                 // column index inside H, if in H
        const bool inH = (jh >= 0 && jh < m);
        if (inH && jh <= k) continue;          // finished columns of H
        const int ilast = inH ? jh : m - 1;    // H: upper triangle only
        const T gkj = G[k * ldg + j] * inv;
        for (int i = k + 1 + ph; i <= ilast; i += tpc)
          G[i * ldg + j] = fma(-G[k * ldg + h0 + i], gkj, G[i * ldg + j]);
      }
    }
    __syncthreads();
  }
}

// After ldl_forward (and a barrier): divide row k by sqrt(d[k]) so that the H
// block's upper triangle becomes L' (L the lower Cholesky factor) and the other
// columns become L^{-1} X.
template <typename T>
LQR_DEV void ldl_scale(T* G, int ldg, int m, int ncols, int h0, const T* d) {
  for (int e = threadIdx.x; e < m * ncols; e += kThreads) {
    const int k = e / ncols, j = e - k * ncols;
    const int jh = j - h0;
    if (jh >= 0 && jh < k) continue;
    G[k * ldg + j] *= T(1) / sqrt(d[k]);
  }
}

// Solve L' X = Z in place for the columns [c0, c1) of G, where L' is the upper
// triangle of the H block (after ldl_scale) and Z the current column content.
// One thread per column walks the triangle (no barriers inside).
template <typename T>
LQR_DEV void ltrsv_cols(T* G, int ldg, int m, int h0, int c0, int c1) {
  for (int j = c0 + threadIdx.x; j < c1; j += kThreads) {
    for (int k = m - 1; k >= 0; --k) {
      T s = G[k * ldg + j];
      for (int l = k + 1; l < m; ++l) s = fma(-G[k * ldg + h0 + l], G[l * ldg + j], s);
      G[k * ldg + j] = s / G[k * ldg + h0 + k];
    }
  }
}

}  // namespace lqr
