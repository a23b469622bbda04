// HISQ staggered hopping stencil (sec. 2.2, eq. 4): one-hop fat link V and
// three-hop long (Naik) link W, for FP64 / FP32 / FP16 storage.
//
// The links stored on the device already carry 1/2 * eta_mu(x) * (time
// boundary sign) (applied when the fields are loaded), so for output parity p
//   hop(x) = sum_mu [V(x) chi(x+mu) - V^dag(x-mu) chi(x-mu)
//                    + W(x) chi(x+3mu) - W^dag(x-3mu) chi(x-3mu)]
// reads chi on parity 1-p only (both hops are odd).  eta_mu does not depend on
// x_mu, so the phase folded into the link at its base site serves the forward
// and the backward hop.  Epilogues:
//   SEPI_HOP   out = k hop
//   SEPI_XPAY  out = a_col x + k hop      (D = m + hop; M_e = m^2 - D_eo D_oe)
// FP16 links are stored divided by one FP32 scale per field (fat, long).
#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

template <int P, int MU, typename R>
__device__ __forceinline__ void stag_dir(const StagArgs& A, const int c[4], int par, int cb, int col,
                                         cx<R>* af, cx<R>* al) {
  const Geom& g = A.g;
  const int pin = par ^ 1;
  const int64_t bi = blk_index(A.in, col, pin);
  cx<R> U[9], x[3], y[3];
  {
    const int nb = nb_cb(c, MU, 1, g);
    IO<P, 3>::load(A.in, bi, nb, x);
    load_link<P, 9>(A.fat, g.Vh, par, MU, cb, U);
    su3_mv(U, x, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) af[a] = af[a] + y[a];
  }
  {
    const int nb = nb_cb(c, MU, -1, g);
    IO<P, 3>::load(A.in, bi, nb, x);
    load_link<P, 9>(A.fat, g.Vh, pin, MU, nb, U);
    su3_mv_dag(U, x, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) af[a] = af[a] - y[a];
  }
  {
    const int nb = nb_cb(c, MU, 3, g);
    IO<P, 3>::load(A.in, bi, nb, x);
    load_link<P, 9>(A.lng, g.Vh, par, MU, cb, U);
    su3_mv(U, x, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) al[a] = al[a] + y[a];
  }
  {
    const int nb = nb_cb(c, MU, -3, g);
    IO<P, 3>::load(A.in, bi, nb, x);
    load_link<P, 9>(A.lng, g.Vh, pin, MU, nb, U);
    su3_mv_dag(U, x, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) al[a] = al[a] - y[a];
  }
}

template <int P, int EPI>
__global__ void __launch_bounds__(256) stag_kernel(StagArgs A) {
  using R = typename RealOf<P>::T;
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  const int ntile = (nsite + blockDim.x - 1) / blockDim.x;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = lb / A.ncol;
  const int col = lb % A.ncol;
  const int j = tile * blockDim.x + threadIdx.x;
  if (tile >= ntile || j >= nsite) return;
  int par, cb;
  if (A.par_out == 2) {
    par = j >= A.g.Vh;
    cb = j - par * A.g.Vh;
  } else {
    par = A.par_out;
    cb = j;
  }
  int c[4];
  cb_coords(cb, par, A.g, c);
  cx<R> af[3] = {{0, 0}, {0, 0}, {0, 0}}, al[3] = {{0, 0}, {0, 0}, {0, 0}};
  stag_dir<P, 0>(A, c, par, cb, col, af, al);
  stag_dir<P, 1>(A, c, par, cb, col, af, al);
  stag_dir<P, 2>(A, c, par, cb, col, af, al);
  stag_dir<P, 3>(A, c, par, cb, col, af, al);
  const R kf = (R)(A.k_hop * A.sfat), kl = (R)(A.k_hop * A.slong);
  cx<R> out[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = kf * af[a] + kl * al[a];
  if constexpr (EPI == SEPI_XPAY) {
    cx<R> x[3];
    IO<P, 3>::load(A.x, blk_index(A.x, col, par), cb, x);
    const R a = A.acol ? (R)A.acol[col] : (R)A.a;
#pragma unroll
    for (int i = 0; i < 3; ++i) out[i] = a * x[i] + out[i];
  }
  IO<P, 3>::store(A.out, blk_index(A.out, col, par), cb, out);
}

int launch_stag(const StagArgs& A, hipStream_t s) {
  const int bs = A.block > 0 ? A.block : 128;
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  const int ntile = (nsite + bs - 1) / bs;
  dim3 grid(ntile * A.ncol), block(bs);
#define LQ_SL(PP)                                                                    \
  if (A.epi == SEPI_HOP) stag_kernel<PP, SEPI_HOP><<<grid, block, 0, s>>>(A);          \
  else stag_kernel<PP, SEPI_XPAY><<<grid, block, 0, s>>>(A);
  if (A.prec == 64) { LQ_SL(64) }
  else if (A.prec == 32) { LQ_SL(32) }
  else { LQ_SL(16) }
#undef LQ_SL
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq
