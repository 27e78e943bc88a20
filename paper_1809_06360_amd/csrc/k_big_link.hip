// Linking solve of the large-state path (65..128 states), FP64, in
// logarithmic depth: the suffix scan of the segment summaries of
// k_link_tree.hip with a join written for 512-thread workgroups. With
// M = I + P0_b Psi_a inverted in place (Gauss-Jordan, partial pivoting,
// big::gj_invert) as E = M^{-1}, F = Gam_a E, U = E'(Psi_a Gam_b):
//   P0_ab = P0_a + (F P0_b) Gam_a',   pbar_ab = pbar_a + F (P0_b psi_a + pbar_b),
//   Gam_ab = F Gam_b,                 Psi_ab = Psi_b + Gam_b' U,
//   psi_ab = psi_b + Gam_b' E'(psi_a - Psi_a pbar_b),
// which is the join of k_link_tree.hip with [X1 | x2 | X3] = E[P0_b Gam_a' |
// P0_b psi_a + pbar_b | Gam_b] multiplied out. The link maps and the forward
// chain of boundary states follow as there.
#include "big_linalg.h"
#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

namespace {

using big::bgemv;
using big::bgemv_t;
using big::bmm1;
using big::kBT;

LQR_DEV double* elem(const double* buf, int n, int j) {
  return const_cast<double*>(buf) + (size_t)j * seg_stride(n);
}

// LDS after the product panels: the inverse's exchange space, vectors, pivot maps.
struct LinkL {
  double *xb, *w1, *w2, *e2;
  int *rowof, *flag;
};

LQR_DEV LinkL carve_link(double* smem) {
  LinkL s;
  s.xb = smem + big::kPanelBytes / sizeof(double);
  s.w1 = s.xb + 512;
  s.w2 = s.w1 + 128;
  s.e2 = s.w2 + 128;
  s.rowof = reinterpret_cast<int*>(s.e2 + 128);
  s.flag = s.rowof + 256;
  return s;
}

}  // namespace

// One scan round: out[j] = in[j] (x) in[j + dist], or in[j] when j + dist >= J.
__global__ __launch_bounds__(kBT) void k_big_link_combine(InstDesc d, int dist, const double* in,
                                                          double* out) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, j = blockIdx.x, nn = n * n;
  const double* a = elem(in, n, j);
  double* o = elem(out, n, j);
  if (j + dist >= J) {
    for (int e = threadIdx.x; e < nn; e += kBT) o[e] = a[e];
    for (int i = threadIdx.x; i < n; i += kBT) o[3 * nn + i] = a[3 * nn + i];
    return;
  }
  const double* b = elem(in, n, j + dist);
  const bool exact_b = j + 2 * dist - 1 >= J - 1;
  const double *P0a = a, *Ga = a + nn, *Psa = a + 2 * nn, *pa = a + 3 * nn, *psa = pa + n;
  const double *P0b = b, *Gb = b + nn, *Psb = b + 2 * nn, *pb = b + 3 * nn, *psb = pb + n;
  double *oP0 = o, *oG = o + nn, *oPs = o + 2 * nn, *op = o + 3 * nn, *ops = op + n;
  const LinkL s = carve_link(smem);
  double* F = big_join_ws(d.ws, n, d.m, J, j);
  double* G1 = F + nn;
  double* V = G1 + nn;
  double* U = V + nn;
  double* E = U + nn;  // M, then M^{-1} (row-major, leading dimension ld)
  const int ld = n;
  if (threadIdx.x == 0) *s.flag = 0;
  // M = I + P0_b Psi_a (P0_b symmetric: read transposed for coalesced loads)
  bmm1<1, true, false, kBT>(n, n, n, P0b, n, Psa, n,
                       [=](int i, int c, double v) { E[i * ld + c] = v + (i == c ? 1.0 : 0.0); });
  __syncthreads();
  big::gj_invert(E, ld, n, s.xb, s.rowof, s.flag);
  double* w1 = s.w1;
  double* w2 = s.w2;
  double* e2 = s.e2;
  bmm1<1, false, false, kBT>(n, n, n, Ga, n, E, ld, [=](int i, int c, double v) { F[i * n + c] = v; });
  bgemv(n, n, P0b, n, psa, [=](int i, double v) { w1[i] = pb[i] + v; });
  if (!exact_b) {
    bmm1<1, true, false, kBT>(n, n, n, Psa, n, Gb, n, [=](int i, int c, double v) { V[i * n + c] = v; });
    bgemv(n, n, Psa, n, pb, [=](int i, double v) { w2[i] = psa[i] - v; });
  }
  __syncthreads();
  bmm1<1, false, false, kBT>(n, n, n, F, n, P0b, n, [=](int i, int c, double v) { G1[i * n + c] = v; });
  bgemv(n, n, F, n, w1, [=](int i, double v) { op[i] = pa[i] + v; });
  if (!exact_b) {
    bmm1<1, false, false, kBT>(n, n, n, F, n, Gb, n, [=](int i, int c, double v) { oG[i * n + c] = v; });
    bmm1<1, true, false, kBT>(n, n, n, E, ld, V, n, [=](int i, int c, double v) { U[i * n + c] = v; });
    bgemv_t(n, n, E, ld, w2, s.xb, [=](int c, double v) { e2[c] = v; });
  }
  __syncthreads();
  bmm1<1, false, true, kBT>(n, n, n, G1, n, Ga, n,
      [=](int i, int c, double v) {
        if (i >= c) {
          v += 0.5 * (P0a[i * n + c] + P0a[c * n + i]);
          oP0[i * n + c] = v;
          oP0[c * n + i] = v;
        }
      },
      SkipUpper{n});
  if (!exact_b) {
    bmm1<1, true, false, kBT>(n, n, n, Gb, n, U, n,
        [=](int i, int c, double v) {
          if (i >= c) {
            v += 0.5 * (Psb[i * n + c] + Psb[c * n + i]);
            oPs[i * n + c] = v;
            oPs[c * n + i] = v;
          }
        },
        SkipUpper{n});
    bgemv_t(n, n, Gb, n, e2, s.xb, [=](int c, double v) { ops[c] = psb[c] + v; });
  }
  __syncthreads();
  if (threadIdx.x == 0 && *s.flag) atomicMax(d.fail + J, LQR_INFO_COUPLING + j);
}

// Boundary values from the scan result and the link maps
//   [F_j | f_j] = N^{-1}[Gam_j' | psi_j - Psi_j p_{t_{j+1}}],  N = I + Psi_j P_{t_{j+1}}.
__global__ __launch_bounds__(kBT) void k_big_link_maps(InstDesc d, const double* fin) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, j = blockIdx.x, nn = n * n;
  {
    const double* sc = elem(fin, n, j);
    double* bnd = ws_bnd(d.ws, n, J, j);
    for (int e = threadIdx.x; e < nn; e += kBT) bnd[e] = sc[e];
    for (int i = threadIdx.x; i < n; i += kBT) bnd[nn + i] = sc[3 * nn + i];
  }
  if (j >= J - 1) return;
  const double* nx = elem(fin, n, j + 1);
  const double *Pn = nx, *pn = nx + 3 * nn;
  const double* sg = ws_seg(d.ws, n, j);
  const double *Gam = sg + nn, *Psi = sg + 2 * nn, *psi = sg + 3 * nn + n;
  const LinkL s = carve_link(smem);
  double* E = big_join_ws(d.ws, n, d.m, J, j) + 4 * (size_t)nn;  // N, then N^{-1}
  const int ld = n;
  double* w = s.w1;
  if (threadIdx.x == 0) *s.flag = 0;
  bmm1<1, true, false, kBT>(n, n, n, Psi, n, Pn, n,
                       [=](int i, int c, double v) { E[i * ld + c] = v + (i == c ? 1.0 : 0.0); });
  bgemv(n, n, Psi, n, pn, [=](int i, double v) { w[i] = psi[i] - v; });
  __syncthreads();
  big::gj_invert(E, ld, n, s.xb, s.rowof, s.flag);
  double* lk = ws_link(d.ws, n, J, j);
  bmm1<1, false, true, kBT>(n, n, n, E, ld, Gam, n, [=](int i, int c, double v) { lk[c * n + i] = v; });
  bgemv(n, n, E, ld, w, [=](int i, double v) { lk[nn + i] = v; });
  __syncthreads();
  if (threadIdx.x == 0 && *s.flag) atomicMax(d.fail + J, LQR_INFO_COUPLING + j);
}

// Boundary states x_{t_{j+1}} = F_j x_{t_j} + f_j from x_{t_0} = x0, then the
// instance's info word. Thread t keeps a quarter row of F_j in registers
// (row t/4, columns 32 (t%4) ..) and loads that of F_{j+1} (and f_{j+1}) while
// step j runs; F is column-major, so 16 consecutive rows of a column are one
// load; the four quarter sums meet by quad permutations.
__global__ __launch_bounds__(kBT) void k_big_link_forward(InstDesc d) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, nn = n * n;
  const int t = threadIdx.x, r = t >> 2, q = t & 3, c0 = 32 * q;
  double* sx = smem;  // two state buffers of 128; entries past n stay zero
  for (int i = t; i < 256; i += kBT) {
    const double v = (i & 127) < n && i < 128 ? d.x0[i] : 0.0;
    sx[i] = v;
    if (i < n) ws_bnd(d.ws, n, J, 0)[nn + n + i] = v;
  }
  // F_jj's quarter row and f_jj's entry of this thread; columns past n load a
  // clamped (finite) element that meets a zero state entry, so no load or
  // product is conditional
  double cur[32], nxt[32], fc = 0.0, fnx = 0.0;
  const int rr = r < n ? r : 0;
  auto fetch = [&](double (&dst)[32], double& fv, int jj) {
    const double* F = ws_link(d.ws, n, J, jj);
#pragma unroll
    for (int c = 0; c < 32; ++c) dst[c] = F[(size_t)min(c0 + c, n - 1) * n + rr];
    fv = F[nn + rr];
  };
  if (J > 1) fetch(cur, fc, 0);
  __syncthreads();
  int b = 0;
  for (int j = 0; j < J - 1; ++j) {
    if (j + 1 < J - 1) fetch(nxt, fnx, j + 1);
    const double* x = sx + b * 128 + c0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c & 3] = fma(cur[c], x[c], acc[c & 3]);
    double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    s += quad_xor<0xB1>(s);  // the four quarter rows of row r
    s += quad_xor<0x4E>(s);
    if (q == 0 && r < n) {
      const double v = s + fc;
      sx[(1 - b) * 128 + r] = v;
      ws_bnd(d.ws, n, J, j + 1)[nn + n + r] = v;
    }
    __syncthreads();
    b = 1 - b;
#pragma unroll
    for (int c = 0; c < 32; ++c) cur[c] = nxt[c];
    fc = fnx;
  }
  if (t == 0) {
    int f = 0;
    for (int jj = 0; jj < J; ++jj) f = combine_info(f, d.fail[jj]);
    *d.info = f ? f : d.fail[J];
  }
}

hipError_t launch_big_link(const InstDesc& d, size_t lds, hipStream_t stream) {
  const int J = d.J, n = d.n;
  hipError_t e = launch_link_init(d, stream);
  if (e != hipSuccess) return e;
  if ((e = ensure_dynamic_lds((const void*)&k_big_link_combine, lds)) != hipSuccess) return e;
  if ((e = ensure_dynamic_lds((const void*)&k_big_link_maps, lds)) != hipSuccess) return e;
  int src = 0;
  for (int dist = 1; dist < J; dist *= 2) {
    const double* in = ws_scan(d.ws, n, J, src);
    double* out = ws_scan(d.ws, n, J, 1 - src);
    hipLaunchKernelGGL(k_big_link_combine, dim3(J), dim3(kBT), lds, stream, d, dist, in, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    src = 1 - src;
  }
  const double* fin = ws_scan(d.ws, n, J, src);
  hipLaunchKernelGGL(k_big_link_maps, dim3(J), dim3(kBT), lds, stream, d, fin);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_link_forward, dim3(1), dim3(kBT), 256 * sizeof(double), stream, d);
  return hipGetLastError();
}

}  // namespace lqr
