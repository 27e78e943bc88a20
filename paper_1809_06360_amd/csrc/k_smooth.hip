// Seeds of the smoothed policies (Sec. III-A): after the linking solve, the
// value at the start of each inner segment k = 1..J-2 is replaced by that
// segment's cost-to-go with its end fixed at its link point z = x_{t_{k+1}}:
// maximising V(x; mu) - mu'z over the end-state price of the segment summary
// V(x; mu) = 1/2 x'P0 x + (Gam mu + pbar)'x + psi'mu - 1/2 mu'Psi mu gives
//   Vxx = P0 + Gam Psi^{-1} Gam',   vx = pbar + Gam Psi^{-1} (psi - z).
// Phase 3 then rebuilds segment k-1 from it instead of the exact value.
// One workgroup per inner segment.
#include "lqr_device.h"
#include "lqr_launch.h"

namespace lqr {

template <int MN, int E>
__global__ __launch_bounds__(kThreads) void k_smooth_seed(InstDesc d) {
  extern __shared__ double smem[];
  const int n = d.n, J = d.J, k = blockIdx.x + 1;
  const int nn = n * n, L = ld_odd(n), blk = n * L;
  const double* sg = ws_seg(d.ws, n, k);
  const double *P0 = sg, *Gam = sg + nn, *Psi = sg + 2 * nn, *pbar = sg + 3 * nn, *psi = pbar + n;
  const double* z = ws_bnd(d.ws, n, J, k + 1) + nn + n;
  double* out = ws_bnd(d.ws, n, J, k);
  double* sPsi = smem;     // Psi (symmetric: row- and column-major alike) -> its inverse
  double* sG = sPsi + blk; // Gam
  double* sT = sG + blk;   // Gam Psi^{-1}
  double* sw = sT + blk;   // psi - z
  const InvExchange ix = carve_inv_exchange(sw + n);
  load_block(sPsi, L, Psi, n, n, n);
  load_block(sG, L, Gam, n, n, n);
  for (int i = threadIdx.x; i < n; i += kThreads) sw[i] = psi[i] - z[i];
  const int bad = wg_invert<MN>(sPsi, L, n, sPsi, L, ix);
  constexpr int E64 = fp64_engine(E);
  pgemm_sub<E64, false, true, false, false>(n, n, n, sG, L, sPsi, L, 0, sG, L, sPsi, L,
      [=](int i, int c, double v) { sT[i * L + c] = v; });
  __syncthreads();
  pgemm_sub<E64, false, true, false, false>(n, n, n, sT, L, sG, L, 0, sT, L, sG, L,
      [=](int i, int c, double v) {
        if (i >= c) {
          v += 0.5 * (P0[i * n + c] + P0[c * n + i]);
          out[i * n + c] = v;
          out[c * n + i] = v;
        }
      },
      SkipUpper{n});
  gemv_wave(1, n, n, sT, L, sw, [=](int i, double v) { out[nn + i] = pbar[i] + v; });
  if (threadIdx.x == 0 && bad) report_info(d.info, LQR_INFO_COUPLING + k);
}

template <int W, int M>
struct k_smooth_seed_ref {
  static auto fn() { return &k_smooth_seed<W, M>; }
};

hipError_t launch_smooth_seed(const InstDesc& d, size_t lds, hipStream_t stream) {
  if (d.J < 3) return hipSuccess;
  return with_link_variant<k_smooth_seed_ref>(d.n, [&](auto kern) -> hipError_t {
    hipError_t e = ensure_dynamic_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(d.J - 2), dim3(kThreads), lds, stream, d);
    return hipGetLastError();
  });
}

}  // namespace lqr
