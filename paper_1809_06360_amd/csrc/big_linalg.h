// Workgroup linear algebra of the large-state kernels (65..128 states, up to
// 64 inputs), for gfx950: 512-thread workgroups (8 wave64s, two per SIMD), so
// that each SIMD has a second wave to issue while the first waits on memory.
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

#include "lqr_layout.h"
#include "wg_linalg.h"

namespace lqr {
namespace big {

constexpr int kBT = 512;        // threads of a large-state workgroup
constexpr int kBW = kBT / 64;   // waves

LQR_DEV int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

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

// One operand stream of a 32x32 block: KC k-steps (4 k each) of the two A
// fragments (rows ia[0], ia[1]) and the two B fragments (columns jb[0], jb[1])
// loaded up front, then 4 KC MFMAs into the 2x2 accumulators. Indices are
// clamped into the operands, out-of-range elements enter as zero.
template <int E, bool TA, bool TB, int KC, typename PA, typename PB>
LQR_DEV void bmm_chunk(typename Mfma<E>::V (&acc)[2][2], const PA* A, int lda, const PB* B, int ldb,
                       int K, const int (&ia)[2], const bool (&iok)[2], const int (&jb)[2],
                       const bool (&jok)[2], int k0, int lk, typename Mfma<E>::T sgn) {
  using T = typename Mfma<E>::T;
  T a[2][KC], b[2][KC];
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    const int k = k0 + 4 * s + lk;
    const bool kin = k < K;
    const int kk = kin ? k : K - 1;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const T va = (T)el<TA>(A, lda, ia[u], kk);
      const T vb = (T)el<TB>(B, ldb, kk, jb[u]);
      a[u][s] = (kin && iok[u]) ? sgn * va : T(0);
      b[u][s] = (kin && jok[u]) ? vb : T(0);
    }
  }
#pragma unroll
  for (int s = 0; s < KC; ++s)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) acc[u][v] = Mfma<E>::op(a[u][s], b[v][s], acc[u][v]);
}

// Matrix-core product of the large-state kernels:
//   v(i, j) = sum_k op(A1)(i,k) op(B1)(k,j) - sum_k op(A2)(i,k) op(B2)(k,j)
// for 0 <= i < M, 0 <= j < N, handed to epi(i, j, v) (v widened to double).
// Each wave takes every kBW-th 32x32 block (2x2 tiles of 16x16, so each
// operand fragment feeds two MFMAs); `skip(i0, j0, 32, 32)` may drop blocks.
template <int E, bool TA1, bool TB1, bool TA2, bool TB2, typename PA1, typename PB1, typename PA2,
          typename PB2, typename Epi, typename Skip = NoSkip>
LQR_DEV void bmm(int M, int N, int K1, const PA1* A1, int lda1, const PB1* B1, int ldb1, int K2,
                 const PA2* A2, int lda2, const PB2* B2, int ldb2, Epi epi, Skip skip = Skip()) {
  using T = typename Mfma<E>::T;
  using V = typename Mfma<E>::V;
  constexpr int KC = 4;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int li = lane & 15, lk = lane >> 4;
  const int nbn = (N + 31) >> 5;
  const int nb = ((M + 31) >> 5) * nbn;
  for (int blk = wave; blk < nb; blk += kBW) {
    const int i0 = (blk / nbn) << 5, j0 = (blk % nbn) << 5;
    if (skip(i0, j0, 32, 32)) continue;
    V acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) acc[u][v] = V{};
    int ia[2], jb[2];
    bool iok[2], jok[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ia[u] = i0 + 16 * u + li;
      iok[u] = ia[u] < M;
      ia[u] = iok[u] ? ia[u] : M - 1;
      jb[u] = j0 + 16 * u + li;
      jok[u] = jb[u] < N;
      jb[u] = jok[u] ? jb[u] : N - 1;
    }
    for (int k0 = 0; k0 < K1; k0 += 4 * KC)
      bmm_chunk<E, TA1, TB1, KC>(acc, A1, lda1, B1, ldb1, K1, ia, iok, jb, jok, k0, lk, T(1));
    for (int k0 = 0; k0 < K2; k0 += 4 * KC)
      bmm_chunk<E, TA2, TB2, KC>(acc, A2, lda2, B2, ldb2, K2, ia, iok, jb, jok, k0, lk, T(-1));
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * u + Mfma<E>::row(lk, r), j = j0 + 16 * v + li;
          if (i < M && j < N) epi(i, j, (double)acc[u][v][r]);
        }
  }
}

template <int E, bool TA, bool TB, typename PA, typename PB, typename Epi, typename Skip = NoSkip>
LQR_DEV void bmm1(int M, int N, int K, const PA* A, int lda, const PB* B, int ldb, Epi epi,
                  Skip skip = Skip()) {
  bmm<E, TA, TB, false, false>(M, N, K, A, lda, B, ldb, 0, A, lda, B, ldb, epi, skip);
}

// y(i) = epi(i, sum_l M[i][l] v[l]) for i < rows (M row-major, any memory; v
// in LDS or global). Eight lanes per row, each summing every eighth column,
// then a reduction over the eight lanes.
template <typename PM, typename PV, typename Epi>
LQR_DEV void bgemv(int rows, int cols, const PM* Mx, int ld, const PV* v, Epi epi) {
  const int sub = threadIdx.x & 7;
  // the eight lanes of a row share i, so each shuffle group is fully active
  for (int i = threadIdx.x >> 3; i < rows; i += kBT >> 3) {
    double s = 0.0;
    for (int l = sub; l < cols; l += 8) s = fma((double)Mx[(size_t)i * ld + l], (double)v[l], s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    if (sub == 0) epi(i, s);
  }
}

// y(j) = epi(j, sum_l M[l][j] v[l]) for j < cols: the transposed product,
// one thread per column (consecutive threads read consecutive columns).
template <typename PM, typename PV, typename Epi>
LQR_DEV void bgemv_t(int rows, int cols, const PM* Mx, int ld, const PV* v, Epi epi) {
  for (int j = threadIdx.x; j < cols; j += kBT) {
    double a0 = 0.0, a1 = 0.0;
    int l = 0;
    for (; l + 2 <= rows; l += 2) {
      a0 = fma((double)Mx[(size_t)l * ld + j], (double)v[l], a0);
      a1 = fma((double)Mx[(size_t)(l + 1) * ld + j], (double)v[l + 1], a1);
    }
    if (l < rows) a0 = fma((double)Mx[(size_t)l * ld + j], (double)v[l], a0);
    epi(j, a0 + a1);
  }
}

// Copy rows x cols between any memories with conversion (dst leading ldd).
template <typename D, typename S>
LQR_DEV void bcopy(D* dst, int ldd, const S* src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kBT) {
    const int i = e / cols, j = e - i * cols;
    dst[(size_t)i * ldd + j] = (D)src[(size_t)i * lds + j];
  }
}

template <typename D>
LQR_DEV void bfill(D* dst, int ldd, int rows, int cols, D v, D diag) {
  const int total = rows * cols;
  for (int e = threadIdx.x; e < total; e += kBT) {
    const int i = e / cols, j = e - i * cols;
    dst[(size_t)i * ldd + j] = (i == j) ? diag : v;
  }
}

// ---------------------------------------------------------------------------
// In-place inverse of an n x n matrix (n <= 128) by Gauss-Jordan elimination
// with partial pivoting, FP64, the matrix held in registers: thread t owns
// rows 4 (t / 16) .. +3 and columns 8 (t % 16) .. +7. Pivots are chosen
// without moving rows (pivot of column k: the unused row with the largest
// magnitude in column k, ties to the lowest row); after all n pivots the
// registers hold the inverse with its rows and columns permuted, which the
// write-back undoes. Per pivot: the owners of column k publish it, every wave
// finds the pivot row, its owners publish it, and every thread updates its 32
// elements (two barriers, double-buffered exchange vectors).
//
// Mx: n x n row-major in LDS (leading dimension ld), replaced by its inverse.
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
