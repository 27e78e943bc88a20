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

// Element e of a round's input: the first round (dist == 1) reads the phase-1
// summaries in place (segments j < J-1, and the last segment's exact value
// from its boundary slot, whose linear term sits right after P); later rounds
// read the scan buffer. `poff` returns the offset of the element's pbar.
LQR_DEV const double* round_elem(const InstDesc& d, const double* in, int dist, int e, int& poff) {
  const int n = d.n, J = d.J, nn = n * n;
  poff = 3 * nn;
  if (dist > 1) return scan_elem(const_cast<double*>(in), n, e);
  if (e < J - 1) return ws_seg(d.ws, n, e);
  poff = nn;
  return ws_bnd(d.ws, n, J, J - 1);
}

}  // namespace

// Scan buffer 0: elements j < J-1 are the phase-1 summaries, element J-1 the
// last segment's exact value; the instance's linking flag is cleared (used by
// the large-state linking solve; the scan below reads the summaries in place).
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
  int apo, bpo;
  const double* a = round_elem(d, in, dist, j, apo);
  double* o = scan_elem(out, n, j);
  if (j + dist >= J) {
    for (int e = threadIdx.x; e < nn; e += kThreads) o[e] = a[e];
    for (int i = threadIdx.x; i < n; i += kThreads) o[3 * nn + i] = a[apo + i];
    return;
  }
  const double* b = round_elem(d, in, dist, j + dist, bpo);
  const bool exact_b = j + 2 * dist - 1 >= J - 1;
  const double *P0a = a, *pa = a + apo, *psa = pa + n;
  const double *Psb = b + 2 * nn, *pb = b + bpo, *psb = pb + n;
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
// chain is serial and latency-bound: wave 0 runs it from LDS (lane i takes
// row i of F_j, F column-major so the lanes read consecutive words; the state
// vector is exchanged through LDS with wave-level ordering and the new states
// are kept in LDS), while waves 1..3 write the previous chunk's states out and
// copy the next chunk of S link maps from global memory into the other half of
// a double buffer with coalesced loads; one workgroup barrier per chunk, so a
// global round trip is paid once per S steps instead of once per step.
template <int MN>
__global__ __launch_bounds__(kThreads) void k_link_forward(InstDesc d) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = link_forward_slots(n);
  const size_t ls = link_stride(n);
  const int steps = J - 1;
  double* sx = smem;                           // 64
  double* sst = smem + 64;                     // 2 x S boundary states (64 each)
  double* buf = sst + 2 * (size_t)S * 64;      // 2 x S link maps
  // boundary states of chunk c, written to the workspace by threads t0..
  auto flush_states = [&](int c, int t0, int nt) {
    if (c < 0) return;
    const int cnt = min(S, steps - c * S);
    const double* st = sst + (size_t)(c & 1) * S * 64;
    for (int e = threadIdx.x - t0; e < cnt * n; e += nt) {
      const int u = e / n, i = e - u * n;
      ws_bnd(d.ws, n, J, c * S + u + 1)[n * n + n + i] = st[u * 64 + i];
    }
  };
  auto copy_chunk = [&](int c, int t0, int nt) {  // chunk c by threads t0.. (nt of them)
    const int j0 = c * S, cnt = min(S, steps - j0);
    if (cnt <= 0) return;
    const double* src = ws_link(d.ws, n, J, j0);  // link maps are contiguous
    double* dst = buf + (size_t)(c & 1) * S * ls;
    const size_t total = (size_t)cnt * ls;
    // up to 64 loads in flight per thread, which covers a whole chunk for
    // every n (clamped indices: no branch per load)
    constexpr int U = 64;
    for (size_t e0 = threadIdx.x - t0; e0 < total; e0 += (size_t)U * nt) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = e0 + (size_t)u * nt;
        v[u] = src[e < total ? e : total - 1];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = e0 + (size_t)u * nt;
        if (e < total) dst[e] = v[u];
      }
    }
  };
  const bool row = lane < n;
  const int r = row ? lane : 0;
  if (wave == 0) {  // entries past n stay zero: padding columns contribute nothing
    const double xi0 = row ? d.x0[lane] : 0.0;
    sx[lane] = xi0;
    if (row) ws_bnd(d.ws, n, J, 0)[n * n + n + lane] = xi0;
  }
  copy_chunk(0, 0, kThreads);
  __syncthreads();
  const int chunks = (steps + S - 1) / S;
  for (int c = 0; c < chunks; ++c) {
    if (wave > 0) {
      flush_states(c - 1, 64, kThreads - 64);
      copy_chunk(c + 1, 64, kThreads - 64);
    } else {
      double* st = sst + (size_t)(c & 1) * S * 64;
      const double* slots = buf + (size_t)(c & 1) * S * ls;
      const int cnt = min(S, steps - c * S);
      for (int u = 0; u < cnt; ++u) {
        const double* F = slots + (size_t)u * ls;
        double f[MN];
#pragma unroll
        for (int k = 0; k < MN; ++k) f[k] = F[(k < n ? k : 0) * n + r];
        __builtin_amdgcn_sched_barrier(0);
        // four accumulation chains
        double acc[4] = {F[(size_t)n * n + r], 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < MN; ++k) acc[k & 3] = fma(f[k], sx[k], acc[k & 3]);
        const double xn = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (row) {
          sx[lane] = xn;
          st[u * 64 + lane] = xn;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  flush_states(chunks - 1, 0, kThreads);
  if (threadIdx.x == 0) {
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
  hipError_t e = hipSuccess;
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
    const size_t lds = link_forward_lds(n);
    hipError_t e2 = ensure_dynamic_lds((const void*)k, lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL(k, dim3(1), dim3(kThreads), lds, stream, d);
    return hipGetLastError();
  });
}

}  // namespace lqr
