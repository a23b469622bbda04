// Wilson-type stencil dispatcher (FP64 instantiations) and the site-term
// kernel of the twisted-clover operator.  The stencil templates live in
// wilson_impl.h; FP32 and FP16 instantiations are in wilson32.hip and
// wilson16.hip so that the three precisions compile in parallel.
#include "wilson_impl.h"

namespace lq {

template int launch_wilson_prec<64>(const WilsonArgs& A, int nr, int bs, hipStream_t s);
extern template int launch_wilson_prec<32>(const WilsonArgs& A, int nr, int bs, hipStream_t s);
extern template int launch_wilson_prec<16>(const WilsonArgs& A, int nr, int bs, hipStream_t s);

int launch_wilson(const WilsonArgs& A, hipStream_t s) {
  if (A.prec == 16 && (A.epi == EPI_CLOVINV || A.epi == EPI_XMY_CLOVINV || A.epi == EPI_SITE ||
                       A.epi == EPI_XMY_RTS || A.epi == EPI_CLOVINV_XPAY))
    return -1;
  const int nr = A.nr > 0 ? A.nr : 1;
  if (!traversal_valid(A.g, A.slab)) return -1;
  const int bs = 0;
  int r;
  if (A.prec == 64) r = launch_wilson_prec<64>(A, nr, bs, s);
  else if (A.prec == 32) r = launch_wilson_prec<32>(A, nr, bs, s);
  else r = launch_wilson_prec<16>(A, nr, bs, s);
  if (r) return r;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq

namespace lq {

// Site term (clover + twist) applied alone: out = A x or A^{-1} x per site.
template <int P, bool INV>
__global__ void __launch_bounds__(256) site_kernel(Geom g, const void* clov, const void* clov_inv, double mu_tw,
                                                   FieldRef in, FieldRef out, int par_out, int ncol) {
  using R = typename RealOf<P>::T;
  const int nsite = par_out == 2 ? 2 * g.Vh : g.Vh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nsite * ncol) return;
  const int col = (int)(i / nsite);
  const int j = (int)(i % nsite);
  const int par = par_out == 2 ? (j >= g.Vh) : par_out;
  const int cb = par_out == 2 ? j - par * g.Vh : j;
  cx<R> x[12], y[12];
  IO<P, 12>::load(in, blk_index(in, col, par), cb, x);
  if constexpr (INV) {
    apply_full6<P>(clov_inv, g.Vh, par, 0, cb, x, y);
    apply_full6<P>(clov_inv, g.Vh, par, 1, cb, x + 6, y + 6);
  } else {
    apply_herm6<P>(clov, g.Vh, par, 0, cb, x, y);
    apply_herm6<P>(clov, g.Vh, par, 1, cb, x + 6, y + 6);
    const R mu = (R)mu_tw;
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = y[k] + mu * times_i(x[k]);
#pragma unroll
    for (int k = 6; k < 12; ++k) y[k] = y[k] - mu * times_i(x[k]);
  }
  IO<P, 12>::store(out, blk_index(out, col, par), cb, y);
}

int launch_site(const Geom& g, int prec, const void* clov, const void* clov_inv, double mu_tw, bool inverse,
                FieldRef in, FieldRef out, int par_out, int ncol, hipStream_t s) {
  const int nsite = par_out == 2 ? 2 * g.Vh : g.Vh;
  const int64_t n = (int64_t)nsite * ncol;
  if (n == 0) return 0;
  const int bs = 256;
  const int nb = (int)((n + bs - 1) / bs);
  if (prec == 64) {
    if (inverse) site_kernel<64, true><<<nb, bs, 0, s>>>(g, clov, clov_inv, mu_tw, in, out, par_out, ncol);
    else site_kernel<64, false><<<nb, bs, 0, s>>>(g, clov, clov_inv, mu_tw, in, out, par_out, ncol);
  } else if (prec == 32) {
    if (inverse) site_kernel<32, true><<<nb, bs, 0, s>>>(g, clov, clov_inv, mu_tw, in, out, par_out, ncol);
    else site_kernel<32, false><<<nb, bs, 0, s>>>(g, clov, clov_inv, mu_tw, in, out, par_out, ncol);
  } else {
    return -8;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq
