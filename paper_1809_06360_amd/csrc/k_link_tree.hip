// Phase 2 in logarithmic depth: the linking solve as a suffix scan of the
// segment summaries under their associative composition.
//
// A segment summary S = (P0, Gam, Psi, pbar, psi) describes the segment's
// cost-to-go as a function of its start state x and of a linear price mu on its
// end state (the dual form of the endpoint-constrained subproblem of Sec. II-A):
//   V(x; mu) = 1/2 x'P0 x + (Gam mu + pbar)'x + psi'mu - 1/2 mu'Psi mu,
// with end state dV/dmu = Gam'x + psi - Psi mu. Joining segment a to the
// segment b that follows it (minimising over the shared boundary state) gives
// a summary of the same form; with M = I + P0_b Psi_a and
//   [X1 | x2 | X3] = M^{-1} [P0_b Gam_a' | P0_b psi_a + pbar_b | Gam_b]:
//   P0_ab = P0_a + Gam_a X1,          pbar_ab = pbar_a + Gam_a x2,
//   Gam_ab = Gam_a X3,                Psi_ab = Psi_b + X3' Psi_a Gam_b,
//   psi_ab = psi_b + X3'(psi_a - Psi_a pbar_b)
// (M' = I + Psi_a P0_b, so X3' = Gam_b' M'^{-1}). The last segment carries
// the terminal cost and no price: its summary is its exact value
// (P0, pbar) = (P, p) at its start with Gam = Psi = psi = 0, and a join
// with such an "exact" b is exact again. The suffix products
// S_j (x) S_{j+1} (x) ... (x) S_{J-1} are therefore the exact value functions at
// the segment boundaries: the quantities the link equation of Sec. II-A
// eliminates one boundary at a time, here found in ceil(log2 J) rounds of
// J - dist independent joins (a Kogge-Stone scan, one workgroup per element).
// The link maps x_{t_{j+1}} = F_j x_{t_j} + f_j then follow in parallel, and a
// last kernel runs the short forward chain of boundary states.
#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

namespace {

LQR_DEV double* scan_elem(double* buf, int n, int j) { return buf + (size_t)j * seg_stride(n); }

}  // namespace

// Scan buffer 0: elements j < J-1 are the phase-1 summaries, element J-1 the
// last segment's exact value; the instance's linking flag is cleared.
__global__ __launch_bounds__(kThreads) void k_link_init(InstDesc d) {
  const int n = d.n, J = d.J, j = blockIdx.x;
  double* dst = scan_elem(ws_scan(d.ws, n, J, 0), n, j);
  if (j < J - 1) {
    const double* src = ws_seg(d.ws, n, j);
    for (size_t e = threadIdx.x; e < seg_stride(n); e += kThreads) dst[e] = src[e];
  } else {
    const double* b = ws_bnd(d.ws, n, J, J - 1);
    for (int e = threadIdx.x; e < n * n; e += kThreads) dst[e] = b[e];
    for (int i = threadIdx.x; i < n; i += kThreads) dst[3 * n * n + i] = b[n * n + i];
  }
  if (j == 0 && threadIdx.x == 0) d.fail[J] = 0;
}

// One scan round: out[j] = in[j] (x) in[j + dist], or in[j] when j + dist >= J
// (then in[j] already reaches the last segment and only its P0, pbar are used).
// The join works from the explicit inverse Mi = M^{-1} (see wg_invert) and
// the identities X1 = Mi P0_b Gam_a', X3 = Mi Gam_b and
// Mi' Psi_a = Psi_a Mi (so V = Psi_a Mi is symmetric):
//   P0_ab  = P0_a + Y R,      Y = Gam_a Mi,  R = P0_b Gam_a'
//   pbar_ab = pbar_a + Gam_a Mi (P0_b psi_a + pbar_b)
//   Gam_ab = Y Gam_b,         Psi_ab = Psi_b + Gam_b' (V Gam_b)
//   psi_ab = psi_b + Gam_b' Mi' (psi_a - Psi_a pbar_b)
// Work blocks in LDS are n x ld_odd(n); row-major unless noted.
template <int MN, int E>
__global__ __launch_bounds__(kThreads) void k_link_combine(InstDesc d, int dist, const double* in,
                                                           double* out) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, j = blockIdx.x;
  const int nn = n * n, L = ld_odd(n), blk = n * L;
  const double* a = scan_elem(const_cast<double*>(in), n, j);
  double* o = scan_elem(out, n, j);
  if (j + dist >= J) {
    for (int e = threadIdx.x; e < nn; e += kThreads) o[e] = a[e];
    for (int i = threadIdx.x; i < n; i += kThreads) o[3 * nn + i] = a[3 * nn + i];
    return;
  }
  const double* b = scan_elem(const_cast<double*>(in), n, j + dist);
  const bool exact_b = j + 2 * dist - 1 >= J - 1;
  const double *P0a = a, *pa = a + 3 * nn, *psa = pa + n;
  const double *Psb = b + 2 * nn, *pb = b + 3 * nn, *psb = pb + n;
  const double *Ga = a + nn, *Psa = a + 2 * nn, *P0b = b, *Gb = b + nn;
  int lg = n;  // leading dimension of the four operands
  double* sM = smem;       // M, column-major -> Mi in place -> U = V Gam_b
  double* sR = sM + blk;   // R = P0_b Gam_a'
  double* sY = sR + blk;   // Y = Gam_a Mi
  double* sV = sY + blk;   // V = Psi_a Mi
  double* r2 = sV + blk;   // P0_b psi_a + pbar_b
  double* sv = r2 + n;     // psi_a - Psi_a pbar_b
  double* su = sv + n;     // Mi' sv
  double* sq = su + n;     // Mi r2
  const InvExchange ix = carve_inv_exchange(sq + n);
  if constexpr (link_tree_staged(MN)) {
    // the four operands, staged in LDS by coalesced loads
    double* st = sq + n + kInvExchangeDoubles;
    double *sGa = st, *sPsa = st + blk, *sP0b = st + 2 * blk, *sGb = st + 3 * blk;
    load_block(sGa, L, Ga, n, n, n);
    load_block(sPsa, L, Psa, n, n, n);
    load_block(sP0b, L, P0b, n, n, n);
    if (!exact_b) load_block(sGb, L, Gb, n, n, n);
    Ga = sGa;
    Psa = sPsa;
    P0b = sP0b;
    Gb = sGb;
    lg = L;
  }
  __syncthreads();
  constexpr int E64 = fp64_engine(E);
  // M = I + P0_b Psi_a (column-major), R = P0_b Gam_a', r2, sv
  pgemm_sub<E64, false, false, false, false>(n, n, n, P0b, lg, Psa, lg, 0, P0b, lg, Psa, lg,
      [=](int i, int c, double v) { sM[c * L + i] = v + (i == c ? 1.0 : 0.0); });
  pgemm_sub<E64, false, true, false, false>(n, n, n, P0b, lg, Ga, lg, 0, P0b, lg, Ga, lg,
      [=](int i, int c, double v) { sR[i * L + c] = v; });
  // P0_b and Psi_a are symmetric: their products walk coalesced columns
  gemv_cm_wave(1, n, n, P0b, lg, psa, [=](int i, double v) { r2[i] = pb[i] + v; });
  if (!exact_b)
    gemv_cm_wave(2, n, n, Psa, lg, pb, [=](int i, double v) { sv[i] = psa[i] - v; });
  const int bad = wg_invert<MN>(sM, L, n, sM, L, ix);
  // Y = Gam_a Mi, V = Psi_a Mi, q = Mi r2, u = Mi' sv
  pgemm_sub<E64, false, true, false, false>(n, n, n, Ga, lg, sM, L, 0, Ga, lg, sM, L,
      [=](int i, int c, double v) { sY[i * L + c] = v; });
  if (!exact_b) {
    pgemm_sub<E64, false, true, false, false>(n, n, n, Psa, lg, sM, L, 0, Psa, lg, sM, L,
        [=](int i, int c, double v) { sV[i * L + c] = v; });
    gemv_wave(1, n, n, sM, L, sv, [=](int i, double v) { su[i] = v; });
  }
  gemv_cm_wave(2, n, n, sM, L, r2, [=](int i, double v) { sq[i] = v; });
  __syncthreads();
  double* oP0 = o;
  double* oG = o + nn;
  double* oPs = o + 2 * nn;
  double* op = o + 3 * nn;
  double* ops = op + n;
  // P0_ab = P0_a + Y R (lower half, mirrored), pbar_ab = pbar_a + Gam_a q
  pgemm_sub<E64, false, false, false, false>(n, n, n, sY, L, sR, L, 0, sY, L, sR, L,
      [=](int i, int c, double v) {
        if (i >= c) {
          v += 0.5 * (P0a[i * n + c] + P0a[c * n + i]);
          oP0[i * n + c] = v;
          oP0[c * n + i] = v;
        }
      },
      SkipUpper{n});
  gemv_wave(1, n, n, Ga, lg, sq, [=](int i, double v) { op[i] = pa[i] + v; });
  if (!exact_b) {
    // Gam_ab = Y Gam_b, U = V Gam_b (into sM: Mi is no longer read),
    // psi_ab = psi_b + Gam_b' u
    pgemm_sub<E64, false, false, false, false>(n, n, n, sY, L, Gb, lg, 0, sY, L, Gb, lg,
        [=](int i, int c, double v) { oG[i * n + c] = v; });
    pgemm_sub<E64, false, false, false, false>(n, n, n, sV, L, Gb, lg, 0, sV, L, Gb, lg,
        [=](int i, int c, double v) { sM[i * L + c] = v; });
    gemv_cm_wave(2, n, n, Gb, lg, su, [=](int i, double v) { ops[i] = psb[i] + v; });
    __syncthreads();
    // Psi_ab = Psi_b + Gam_b' U (lower half, mirrored)
    pgemm_sub<E64, true, false, false, false>(n, n, n, Gb, lg, sM, L, 0, Gb, lg, sM, L,
        [=](int i, int c, double v) {
          if (i >= c) {
            v += 0.5 * (Psb[i * n + c] + Psb[c * n + i]);
            oPs[i * n + c] = v;
            oPs[c * n + i] = v;
          }
        },
        SkipUpper{n});
  }
  if (threadIdx.x == 0 && bad) atomicMax(d.fail + J, LQR_INFO_COUPLING + j);
}

// Boundary values from the scan result, and the link maps
//   [F_j | f_j] = N^{-1}[Gam_j' | psi_j - Psi_j p_{t_{j+1}}],  N = I + Psi_j P_{t_{j+1}}
// (one workgroup per boundary; the last workgroup only copies its value).
template <int MN, int E>
__global__ __launch_bounds__(kThreads) void k_link_maps(InstDesc d, const double* fin) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, j = blockIdx.x;
  const int nn = n * n, L = ld_odd(n), blk = n * L;
  {
    const double* s = scan_elem(const_cast<double*>(fin), n, j);
    double* bnd = ws_bnd(d.ws, n, J, j);
    for (int e = threadIdx.x; e < nn; e += kThreads) bnd[e] = s[e];
    for (int i = threadIdx.x; i < n; i += kThreads) bnd[nn + i] = s[3 * nn + i];
  }
  if (j >= J - 1) return;
  const double* nx = scan_elem(const_cast<double*>(fin), n, j + 1);
  const double* Pn = nx;
  const double* pn = nx + 3 * nn;
  const double* sg = ws_seg(d.ws, n, j);
  const double *Gam = sg + nn, *Psi = sg + 2 * nn, *psi = sg + 3 * nn + n;
  double* sN = smem;        // N, column-major -> its inverse in place
  double* sG = sN + blk;    // Gam (row-major)
  double* sw = sG + blk;    // psi - Psi pn
  const InvExchange ix = carve_inv_exchange(sw + n);
  constexpr int E64 = fp64_engine(E);
  load_block(sG, L, Gam, n, n, n);
  pgemm_sub<E64, false, false, false, false>(n, n, n, Psi, n, Pn, n, 0, Psi, n, Pn, n,
      [=](int i, int c, double v) { sN[c * L + i] = v + (i == c ? 1.0 : 0.0); });
  // Psi is symmetric: its product walks coalesced columns
  gemv_cm_wave(1, n, n, Psi, n, pn, [=](int i, double v) { sw[i] = psi[i] - v; });
  const int bad = wg_invert<MN>(sN, L, n, sN, L, ix);
  double* lk = ws_link(d.ws, n, J, j);
  // F' = Gam N^{-T} (row c of F' is column c of F: the workspace keeps F
  // column-major, with coalesced stores here), f = N^{-1} w
  pgemm_sub<E64, false, false, false, false>(n, n, n, sG, L, sN, L, 0, sG, L, sN, L,
      [=](int c, int i, double v) { lk[c * n + i] = v; });
  gemv_cm_wave(1, n, n, sN, L, sw, [=](int i, double v) { lk[nn + i] = v; });
  if (threadIdx.x == 0 && bad) atomicMax(d.fail + J, LQR_INFO_COUPLING + j);
}

// Boundary states x_{t_{j+1}} = F_j x_{t_j} + f_j from x_{t_0} = x0, and the
// instance's info word (a stage failure of phase 1 takes precedence). The
// chain is serial and latency-bound, so it runs in one wave: lane i keeps row
// i of F_j in registers (row i of F_{j+1} is loaded while step j computes;
// with F column-major each of those loads is one coalesced column) and the
// state vector is exchanged through LDS with wave-level ordering.
template <int MN>
__global__ __launch_bounds__(64) void k_link_forward(InstDesc d) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, lane = threadIdx.x;
  double* sx = smem;
  const bool row = lane < n;
  const double xi0 = row ? d.x0[lane] : 0.0;
  if (row) {
    sx[lane] = xi0;
    ws_bnd(d.ws, n, J, 0)[n * n + n + lane] = xi0;
  }
  double cur[MN], nxt[MN];
#pragma unroll
  for (int k = 0; k < MN; ++k) nxt[k] = 0.0;
#pragma unroll
  for (int k = 0; k < MN; ++k) cur[k] = 0.0;
  if (J > 1 && row) {
    const double* F = ws_link(d.ws, n, J, 0) + lane;
#pragma unroll
    for (int k = 0; k < MN; ++k) cur[k] = k < n ? F[k * n] : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int j = 0; j < J - 1; ++j) {
    const double* lk = ws_link(d.ws, n, J, j);
    if (j + 1 < J - 1 && row) {
      const double* F = ws_link(d.ws, n, J, j + 1) + lane;
#pragma unroll
      for (int k = 0; k < MN; ++k) nxt[k] = k < n ? F[k * n] : 0.0;
    }
    // four accumulation chains
    double acc[4] = {row ? lk[n * n + lane] : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < MN; ++k) acc[k & 3] = fma(cur[k], sx[k < n ? k : 0], acc[k & 3]);
    const double xn = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (row) {
      sx[lane] = xn;
      ws_bnd(d.ws, n, J, j + 1)[n * n + n + lane] = xn;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < MN; ++k) cur[k] = nxt[k];
  }
  if (lane == 0) {
    int f = 0;
    for (int j = 0; j < J; ++j) f = combine_info(f, d.fail[j]);
    *d.info = f ? f : d.fail[J];
  }
}

template <int W, int M>
struct k_link_forward_ref {
  static auto fn() { return &k_link_forward<W>; }
};

template <int W, int M>
struct k_link_combine_ref {
  static auto fn() { return &k_link_combine<W, M>; }
};
template <int W, int M>
struct k_link_maps_ref {
  static auto fn() { return &k_link_maps<W, M>; }
};

hipError_t launch_link_init(const InstDesc& d, hipStream_t stream) {
  hipLaunchKernelGGL(k_link_init, dim3(d.J), dim3(kThreads), 0, stream, d);
  return hipGetLastError();
}

hipError_t launch_link_tree(const InstDesc& d, size_t lds, hipStream_t stream) {
  const int J = d.J, n = d.n;
  hipLaunchKernelGGL(k_link_init, dim3(J), dim3(kThreads), 0, stream, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int src = 0;
  for (int dist = 1; dist < J; dist *= 2) {
    const double* in = ws_scan(d.ws, n, J, src);
    double* out = ws_scan(d.ws, n, J, 1 - src);
    e = with_link_variant<k_link_combine_ref>(n, [&](auto k) -> hipError_t {
      hipError_t e2 = ensure_dynamic_lds((const void*)k, lds);
      if (e2 != hipSuccess) return e2;
      hipLaunchKernelGGL(k, dim3(J), dim3(kThreads), lds, stream, d, dist, in, out);
      return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    src = 1 - src;
  }
  const double* fin = ws_scan(d.ws, n, J, src);
  e = with_link_variant<k_link_maps_ref>(n, [&](auto k) -> hipError_t {
    hipError_t e2 = ensure_dynamic_lds((const void*)k, lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL(k, dim3(J), dim3(kThreads), lds, stream, d, fin);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return with_link_variant<k_link_forward_ref>(n, [&](auto k) -> hipError_t {
    hipLaunchKernelGGL(k, dim3(1), dim3(64), 64 * sizeof(double), stream, d);
    return hipGetLastError();
  });
}

}  // namespace lqr
