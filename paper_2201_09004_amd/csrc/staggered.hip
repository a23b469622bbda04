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
//   SEPI_XPAY_DOT  the same and <x, out> per column and 64-site tile (CG's
//              <p, M_e p> without a separate pass over p and M_e p)
// FP16 links are stored divided by one FP32 scale per field (fat, long).
// One thread owns one site and NR consecutive columns: the 16 links of a site
// are loaded once for all NR columns (bitwise-identical per-column results
// for every NR), and the NR neighbour loads of a hop are issued together.
// FP16 products are formed by v_dot2_f32_f16 on the packed halves.
#include <type_traits>

#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

template <int P, int MU, int K, bool LONG, int NR, typename R>
__device__ __forceinline__ void stag_hop1(const StagArgs& A, const int c[4], int par, int cb, int col0, int nv,
                                          cx<R> (*acc)[3]) {
  const Geom& g = A.g;
  const int pin = par ^ 1;
  const void* links = LONG ? A.lng : A.fat;
  const int nb = nb_cb(c, MU, K, g);
  if constexpr (P == 16) {
    // FP16 products by v_dot2_f32_f16 (dot2h); the link is rearranged once for
    // all NR columns so that each real part is one dot2h on the neighbour's
    // packed halves x_j = (re, im), and the neighbour's site norm scales the sum:
    //   U x:      re = dot2h((u.re, -u.im), x_j), im = dot2h((u.im, u.re), x_j)
    //   U^dag x:  re = dot2h((u.re, u.im), x_j),  im = dot2h((-u.im, u.re), x_j)
    unsigned Ur[9], Ui[9];
    {
      const unsigned* lp = (const unsigned*)links;
      const int grp = (K > 0 ? par : pin) * 4 + MU;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        const unsigned u = ldx<true>(lp + tix(grp, e, 9, K > 0 ? cb : nb, g.Vh));
        Ur[e] = K > 0 ? u ^ kSignHi : u;
        Ui[e] = K > 0 ? swap_halves(u) : swap_halves(u) ^ kSignLo;
      }
    }
    uint4 xn[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      xn[r] = ldx<false>((const uint4*)A.in.data + tix(blk_index(A.in, min(col0 + r, A.ncol - 1), pin), 0, 1, nb,
                                                      A.in.Vh));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const float n = __uint_as_float(xn[r].w);
      const unsigned w[3] = {xn[r].x, xn[r].y, xn[r].z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float yr = 0.f, yi = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const int e = K > 0 ? 3 * a + j : 3 * j + a;
          yr = dot2h(Ur[e], w[j], yr);
          yi = dot2h(Ui[e], w[j], yi);
        }
        const float sn = K > 0 ? n : -n;
        acc[r][a].re = fmar(sn, yr, acc[r][a].re);
        acc[r][a].im = fmar(sn, yi, acc[r][a].im);
      }
    }
  } else {
    cx<R> U[9];
    if constexpr (K > 0) load_link<P, 9>(links, g.Vh, par, MU, cb, U);
    else load_link<P, 9>(links, g.Vh, pin, MU, nb, U);
    // all NR columns' loads in flight at once (columns past the last are
    // clamped to a valid one and their results dropped)
    cx<R> xn[NR][3];
#pragma unroll
    for (int r = 0; r < NR; ++r) IO<P, 3>::load(A.in, blk_index(A.in, min(col0 + r, A.ncol - 1), pin), nb, xn[r]);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      cx<R> y[3];
      if constexpr (K > 0) {
        su3_mv(U, xn[r], y);
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[r][a] = acc[r][a] + y[a];
      } else {
        su3_mv_dag(U, xn[r], y);
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[r][a] = acc[r][a] - y[a];
      }
    }
  }
}

// Passes the accumulators through an empty asm statement that also clobbers
// memory: the arithmetic before it is done before it, the loads after it are
// issued after it (without it the compiler issues every hop's loads first and
// holds all neighbours in registers).
template <int NR, typename R>
__device__ __forceinline__ void pin3(cx<R> (*a)[3]) {
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i) asm volatile("" : "+v"(a[r][i].re), "+v"(a[r][i].im)::"memory");
}

// the backward (x - mu, x - 3 mu) and the forward (x + mu, x + 3 mu) hops of one direction
template <int P, int MU, int NR, typename R>
__device__ __forceinline__ void stag_back(const StagArgs& A, const int c[4], int par, int cb, int col0, int nv,
                                          cx<R> (*af)[3], cx<R> (*al)[3]) {
  stag_hop1<P, MU, -3, true, NR>(A, c, par, cb, col0, nv, al);
  stag_hop1<P, MU, -1, false, NR>(A, c, par, cb, col0, nv, af);
  pin3<NR>(af);
  pin3<NR>(al);
}
template <int P, int MU, int NR, typename R>
__device__ __forceinline__ void stag_fwd(const StagArgs& A, const int c[4], int par, int cb, int col0, int nv,
                                         cx<R> (*af)[3], cx<R> (*al)[3]) {
  stag_hop1<P, MU, 1, false, NR>(A, c, par, cb, col0, nv, af);
  stag_hop1<P, MU, 3, true, NR>(A, c, par, cb, col0, nv, al);
  pin3<NR>(af);
  pin3<NR>(al);
}

template <int P, int EPI, int NR>
__global__ void __launch_bounds__(kStencilMaxThreads) stag_kernel(StagArgs A) {
  using R = typename RealOf<P>::T;
  constexpr bool RED = EPI == SEPI_XPAY_DOT;
  if (A.ncol <= 0) return;
  const int ngrp = (A.ncol + NR - 1) / NR;
  int par, cb, grp, c[4], tile = 0;
  const int status = stencil_site(A.g, A.par_out, A.slab, ngrp, A.sh, par, cb, grp, c, &tile);
  // lanes past the end of the last tile stay only to join the wave reductions
  if (status == 0 || (!RED && status != 1)) return;
  const bool live = status == 1;
  const int col0 = grp * NR;
  const int nv = min(NR, A.ncol - col0);
  cx<R> af[NR][3], al[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) af[r][a] = al[r][a] = {0, 0};
  // backward hops from t down to x, then forward hops from x up to t: a
  // neighbour read as +mu by one wave is read as -mu by a wave started
  // later, and this order brings the two reads closer in time (L2 hits)
  stag_back<P, 3, NR>(A, c, par, cb, col0, nv, af, al);
  stag_back<P, 2, NR>(A, c, par, cb, col0, nv, af, al);
  stag_back<P, 1, NR>(A, c, par, cb, col0, nv, af, al);
  stag_back<P, 0, NR>(A, c, par, cb, col0, nv, af, al);
  stag_fwd<P, 0, NR>(A, c, par, cb, col0, nv, af, al);
  stag_fwd<P, 1, NR>(A, c, par, cb, col0, nv, af, al);
  stag_fwd<P, 2, NR>(A, c, par, cb, col0, nv, af, al);
  stag_fwd<P, 3, NR>(A, c, par, cb, col0, nv, af, al);
  const R kf = (R)(A.k_hop * A.sfat), kl = (R)(A.k_hop * A.slong);
  double red[NR][2];
#pragma unroll
  for (int r = 0; r < NR; ++r) red[r][0] = red[r][1] = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nv) continue;
    const int col = col0 + r;
    cx<R> out[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = kf * af[r][a] + kl * al[r][a];
    if constexpr (EPI == SEPI_XPAY || EPI == SEPI_XPAY_DOT) {
      cx<R> x[3];
      IO<P, 3>::template load<true>(A.x, blk_index(A.x, col, par), cb, x);
      const R a = A.acol ? (R)A.acol[col] : (R)A.a;
#pragma unroll
      for (int i = 0; i < 3; ++i) out[i] = a * x[i] + out[i];
      if constexpr (RED) {
        if (live) {
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            red[r][0] += (double)x[i].re * (double)out[i].re + (double)x[i].im * (double)out[i].im;
            red[r][1] += (double)x[i].re * (double)out[i].im - (double)x[i].im * (double)out[i].re;
          }
        }
      }
    }
    if (live) IO<P, 3>::template store<true>(A.out, blk_index(A.out, col, par), cb, out);
  }
  if constexpr (RED) {
    // wave butterfly (fixed order) and one partial per (column, 64-site tile)
    const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
    const int ntile = (nsite + 63) >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nv) continue;
#pragma unroll
      for (int k = 0; k < 2; ++k)
        for (int o = 32; o > 0; o >>= 1) red[r][k] += __shfl_xor(red[r][k], o);
      if ((threadIdx.x & 63) == 0) {
        double* q = A.red + ((int64_t)(col0 + r) * ntile + tile) * 4;
        q[0] = red[r][0];
        q[1] = red[r][1];
        q[2] = 0.0;
        q[3] = 0.0;
      }
    }
  }
}

template <int P, int EPI, int NR>
static void stag_one(const StagArgs& A, int bs, hipStream_t s) {
  (void)bs;
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  const StencilGrid G = stencil_grid(nsite, (A.ncol + NR - 1) / NR, A.tpb, A.xcd);
  StagArgs B = A;
  B.sh = G.sh;
  stag_kernel<P, EPI, NR><<<dim3(G.blocks), dim3(G.threads), 0, s>>>(B);
}

template <int P, int EPI>
static int stag_nr(const StagArgs& A, int nr, int bs, hipStream_t s) {
  switch (nr) {
    case 1: stag_one<P, EPI, 1>(A, bs, s); return 0;
    case 2: stag_one<P, EPI, 2>(A, bs, s); return 0;
    case 3: stag_one<P, EPI, 3>(A, bs, s); return 0;
    case 4: stag_one<P, EPI, 4>(A, bs, s); return 0;
    case 6: stag_one<P, EPI, 6>(A, bs, s); return 0;
    case 8: stag_one<P, EPI, 8>(A, bs, s); return 0;
    default: return -1;
  }
}

int launch_stag(const StagArgs& A, hipStream_t s) {
  const int nr = A.nr > 0 ? A.nr : 1;
  if (!traversal_valid(A.g, A.slab)) return -1;
  const int bs = 0;
  int r;
  auto pick = [&](auto p) -> int {
    constexpr int P = decltype(p)::value;
    if (A.epi == SEPI_HOP) return stag_nr<P, SEPI_HOP>(A, nr, bs, s);
    if (A.epi == SEPI_XPAY) return stag_nr<P, SEPI_XPAY>(A, nr, bs, s);
    return stag_nr<P, SEPI_XPAY_DOT>(A, nr, bs, s);
  };
  if (A.prec == 64) r = pick(std::integral_constant<int, 64>{});
  else if (A.prec == 32) r = pick(std::integral_constant<int, 32>{});
  else r = pick(std::integral_constant<int, 16>{});
  if (r) return r;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq
