// Wilson-type hopping stencil (sec. 2.1, eq. 2; sec. 2.3 for H_W) with fused
// epilogues, for FP64 / FP32 / FP16 storage and full or reconstructed links.
//
// For output parity p the kernel computes, per site x and column,
//   hop(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu^dag(x-mu) psi(x-mu)]
// reading psi on parity 1-p (the dagger swaps the two projectors), then one of
//   EPI_HOP        out = k hop
//   EPI_XPAY       out = a x + k hop                 (Wilson D, staggered-free)
//   EPI_XPAY_G5    out = g5 (a x + k hop)            (H_W = g5 D_W(-rho), eq. after 5)
//   EPI_CLOVINV    out = A^{-1} (k hop)              (first half of the Schur operator)
//   EPI_XMY_CLOVINV out = x - A^{-1} (k hop)         (second half)
//   EPI_SITE       out = A x + k hop,  A = H + i mu g5 (full twisted-clover D)
//   EPI_CHEB       out = s1 g5 (a x + k hop) + ck v + s2 b1 - b2   (one Clenshaw step)
// where x, v, b1, b2 are fields of the output parity.  The time-boundary
// sign is applied here from the coordinates, so links stay exactly SU(3)
// for the 12-real reconstruction.
//
// Spin projection in the chiral basis g_mu = [[0, P_mu], [P_mu^dag, 0]],
// P_k = -i sigma_k, P_4 = 1: (1 + s g_mu) psi = (h, s P_mu^dag h) with
// h = psi_up + s P_mu psi_low, so only two colour vectors are multiplied by the link.
#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cx<R>* p, cx<R>* h) {
  const R s = (R)S;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
    if constexpr (MU == 0) {
      h[a] = p0 + s * times_mi(p3);
      h[3 + a] = p1 + s * times_mi(p2);
    } else if constexpr (MU == 1) {
      h[a] = p0 - s * p3;
      h[3 + a] = p1 + s * p2;
    } else if constexpr (MU == 2) {
      h[a] = p0 + s * times_mi(p2);
      h[3 + a] = p1 + s * times_i(p3);
    } else {
      h[a] = p0 + s * p2;
      h[3 + a] = p1 + s * p3;
    }
  }
}

template <int MU, int S, typename R>
__device__ __forceinline__ void recon_add(cx<R>* o, const cx<R>* h) {
  const R s = (R)S;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> h0 = h[a], h1 = h[3 + a];
    o[a] = o[a] + h0;
    o[3 + a] = o[3 + a] + h1;
    if constexpr (MU == 0) {
      o[6 + a] = o[6 + a] + s * times_i(h1);
      o[9 + a] = o[9 + a] + s * times_i(h0);
    } else if constexpr (MU == 1) {
      o[6 + a] = o[6 + a] + s * h1;
      o[9 + a] = o[9 + a] - s * h0;
    } else if constexpr (MU == 2) {
      o[6 + a] = o[6 + a] + s * times_i(h0);
      o[9 + a] = o[9 + a] + s * times_mi(h1);
    } else {
      o[6 + a] = o[6 + a] + s * h0;
      o[9 + a] = o[9 + a] + s * h1;
    }
  }
}

template <int P, int NE, bool DAG, int MU, typename R>
__device__ __forceinline__ void hop_dir(const WilsonArgs& A, const int c[4], int par, int cb, int col,
                                        cx<R>* acc) {
  const Geom& g = A.g;
  const int pin = par ^ 1;
  cx<R> U[9], psi[12], h[6], uh[6];
  // forward: (1 - g) U_mu(x) psi(x + mu); dagger: (1 + g)
  {
    const int nb = nb_cb(c, MU, 1, g);
    IO<P, 12>::load(A.in, blk_index(A.in, col, pin), nb, psi);
    project<MU, DAG ? 1 : -1>(psi, h);
    load_link<P, NE>(A.links, g.Vh, par, MU, cb, U);
    su3_mv(U, h, uh);
    su3_mv(U, h + 3, uh + 3);
    if (MU == 3 && g.ap && c[3] == g.L[3] - 1) {
#pragma unroll
      for (int i = 0; i < 6; ++i) uh[i] = -uh[i];
    }
    recon_add<MU, DAG ? 1 : -1>(acc, uh);
  }
  // backward: (1 + g) U_mu^dag(x - mu) psi(x - mu); dagger: (1 - g)
  {
    const int nb = nb_cb(c, MU, -1, g);
    IO<P, 12>::load(A.in, blk_index(A.in, col, pin), nb, psi);
    project<MU, DAG ? -1 : 1>(psi, h);
    load_link<P, NE>(A.links, g.Vh, pin, MU, nb, U);
    su3_mv_dag(U, h, uh);
    su3_mv_dag(U, h + 3, uh + 3);
    if (MU == 3 && g.ap && c[3] == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) uh[i] = -uh[i];
    }
    recon_add<MU, DAG ? -1 : 1>(acc, uh);
  }
}

// 6x6 complex matrix [36] (row-major) times the chiral half of a spinor
template <int P, typename R>
__device__ __forceinline__ void apply_full6(const void* base, int Vh, int par, int chir, int cb,
                                            const cx<R>* v, cx<R>* y) {
  using T2 = typename LinkT<P>::T2;
  const T2* p = (const T2*)base + ((int64_t)(par * 2 + chir) * 36) * Vh + cb;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    cx<R> s = {0, 0};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      T2 d = p[(int64_t)(i * 6 + j) * Vh];
      fma(s, cx<R>{(R)d.x, (R)d.y}, v[j]);
    }
    y[i] = s;
  }
}

// Hermitian 6x6 packed as 3 T2 of diagonal pairs + 15 lower entries (i>j, row order)
template <int P, typename R>
__device__ __forceinline__ void apply_herm6(const void* base, int Vh, int par, int chir, int cb,
                                            const cx<R>* v, cx<R>* y) {
  using T2 = typename LinkT<P>::T2;
  const T2* p = (const T2*)base + ((int64_t)(par * 2 + chir) * 18) * Vh + cb;
  R d[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T2 e = p[(int64_t)k * Vh];
    d[2 * k] = (R)e.x;
    d[2 * k + 1] = (R)e.y;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] = d[i] * v[i];
  int k = 3;
#pragma unroll
  for (int i = 1; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j < i; ++j) {
      T2 e = p[(int64_t)k * Vh];
      ++k;
      cx<R> l = {(R)e.x, (R)e.y};
      fma(y[i], l, v[j]);
      fmac(y[j], l, v[i]);
    }
  }
}

template <int P, int NE, bool DAG, int EPI>
__global__ void __launch_bounds__(256) wilson_kernel(WilsonArgs A) {
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

  cx<R> acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = {0, 0};
  hop_dir<P, NE, DAG, 0>(A, c, par, cb, col, acc);
  hop_dir<P, NE, DAG, 1>(A, c, par, cb, col, acc);
  hop_dir<P, NE, DAG, 2>(A, c, par, cb, col, acc);
  hop_dir<P, NE, DAG, 3>(A, c, par, cb, col, acc);

  const R k = (R)A.k_hop;
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = k * acc[i];

  cx<R> out[12];
  if constexpr (EPI == EPI_HOP) {
#pragma unroll
    for (int i = 0; i < 12; ++i) out[i] = acc[i];
  } else if constexpr (EPI == EPI_XPAY || EPI == EPI_XPAY_G5 || EPI == EPI_CHEB) {
    cx<R> x[12];
    IO<P, 12>::load(A.x, blk_index(A.x, col, par), cb, x);
    const R a = A.acol ? (R)A.acol[col] : (R)A.a;
#pragma unroll
    for (int i = 0; i < 12; ++i) out[i] = a * x[i] + acc[i];
    if constexpr (EPI != EPI_XPAY) {
#pragma unroll
      for (int i = 6; i < 12; ++i) out[i] = -out[i];
    }
    if constexpr (EPI == EPI_CHEB) {
      cx<R> v[12];
      const R s1 = (R)A.s1, ck = (R)A.ck, s2 = (R)A.s2;
      IO<P, 12>::load(A.v, blk_index(A.v, col, par), cb, v);
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = s1 * out[i] + ck * v[i];
      IO<P, 12>::load(A.b1, blk_index(A.b1, col, par), cb, v);
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = out[i] + s2 * v[i];
      IO<P, 12>::load(A.b2, blk_index(A.b2, col, par), cb, v);
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = out[i] - v[i];
    }
  } else if constexpr (EPI == EPI_CLOVINV || EPI == EPI_XMY_CLOVINV) {
    apply_full6<P>(A.clov_inv, A.g.Vh, par, 0, cb, acc, out);
    apply_full6<P>(A.clov_inv, A.g.Vh, par, 1, cb, acc + 6, out + 6);
    if constexpr (EPI == EPI_XMY_CLOVINV) {
      cx<R> x[12];
      IO<P, 12>::load(A.x, blk_index(A.x, col, par), cb, x);
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = x[i] - out[i];
    }
  } else if constexpr (EPI == EPI_SITE) {
    cx<R> x[12];
    IO<P, 12>::load(A.x, blk_index(A.x, col, par), cb, x);
    apply_herm6<P>(A.clov, A.g.Vh, par, 0, cb, x, out);
    apply_herm6<P>(A.clov, A.g.Vh, par, 1, cb, x + 6, out + 6);
    const R mu = (R)A.mu_tw;
#pragma unroll
    for (int i = 0; i < 6; ++i) out[i] = out[i] + mu * times_i(x[i]) + acc[i];
#pragma unroll
    for (int i = 6; i < 12; ++i) out[i] = out[i] - mu * times_i(x[i]) + acc[i];
  }
  IO<P, 12>::store(A.out, blk_index(A.out, col, par), cb, out);
}

template <int P, int NE, bool DAG>
static void launch_epi(const WilsonArgs& A, dim3 grid, dim3 block, hipStream_t s) {
  switch (A.epi) {
    case EPI_HOP: wilson_kernel<P, NE, DAG, EPI_HOP><<<grid, block, 0, s>>>(A); break;
    case EPI_XPAY: wilson_kernel<P, NE, DAG, EPI_XPAY><<<grid, block, 0, s>>>(A); break;
    case EPI_XPAY_G5: wilson_kernel<P, NE, DAG, EPI_XPAY_G5><<<grid, block, 0, s>>>(A); break;
    case EPI_CHEB: wilson_kernel<P, NE, DAG, EPI_CHEB><<<grid, block, 0, s>>>(A); break;
    default:
      if constexpr (P != 16) {
        switch (A.epi) {
          case EPI_CLOVINV: wilson_kernel<P, NE, DAG, EPI_CLOVINV><<<grid, block, 0, s>>>(A); break;
          case EPI_XMY_CLOVINV: wilson_kernel<P, NE, DAG, EPI_XMY_CLOVINV><<<grid, block, 0, s>>>(A); break;
          case EPI_SITE: wilson_kernel<P, NE, DAG, EPI_SITE><<<grid, block, 0, s>>>(A); break;
        }
      }
  }
}

template <int P>
static void launch_prec(const WilsonArgs& A, dim3 grid, dim3 block, hipStream_t s) {
  if (A.recon && P != 64) {
    if (A.dag) launch_epi<P, 6, true>(A, grid, block, s);
    else launch_epi<P, 6, false>(A, grid, block, s);
  } else {
    if (A.dag) launch_epi<P, 9, true>(A, grid, block, s);
    else launch_epi<P, 9, false>(A, grid, block, s);
  }
}

int launch_wilson(const WilsonArgs& A, hipStream_t s) {
  if (A.prec == 16 && (A.epi == EPI_CLOVINV || A.epi == EPI_XMY_CLOVINV || A.epi == EPI_SITE)) return -1;
  const int bs = A.block > 0 ? A.block : 128;
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  const int ntile = (nsite + bs - 1) / bs;
  dim3 grid(ntile * A.ncol), block(bs);
  if (A.prec == 64) launch_prec<64>(A, grid, block, s);
  else if (A.prec == 32) launch_prec<32>(A, grid, block, s);
  else launch_prec<16>(A, grid, block, s);
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
