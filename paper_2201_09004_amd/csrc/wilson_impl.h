// Wilson-type hopping stencil (sec. 2.1, eq. 2; sec. 2.3 for H_W) with fused
// epilogues, for FP64 / FP32 / FP16 storage and full or reconstructed links.
//
// For output parity p the kernel computes, per site x and column,
//   hop(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu^dag(x-mu) psi(x-mu)]
// reading psi on parity 1-p (the dagger swaps the two projectors), then one of
//   EPI_HOP         out = k hop
//   EPI_XPAY        out = a x + k hop                 (Wilson D)
//   EPI_XPAY_G5     out = g5 (a x + k hop)            (H_W = g5 D_W(-rho), sec. 2.3)
//   EPI_CLOVINV     out = A^{-1} (k hop)              (first half of the Schur operator)
//   EPI_CLOVINV_XPAY out = A^{-1} (x + k hop)         (even-odd source, odd-site reconstruction)
//   EPI_XMY_CLOVINV out = x - A^{-1} (k hop)          (second half)
//   EPI_SITE        out = A x + k hop,  A = H + i mu g5 (full twisted-clover D)
//   EPI_CHEB        out = s1 g5 (a x + k hop) + ck v + s2 b1 - b2   (one Clenshaw step)
// where x, v, b1, b2 are fields of the output parity.  The time-boundary
// sign is applied here from the coordinates, so links stay exactly SU(3)
// for the 12-real reconstruction.
//
// Register blocking: one thread owns one site and NR consecutive columns, so
// each link and each site matrix is loaded once and used NR times.  Every
// column is computed with the same arithmetic in the same order whatever NR
// is, so all NR variants give bitwise-identical results.
//
// Spin projection in the chiral basis g_mu = [[0, P_mu], [P_mu^dag, 0]],
// P_k = -i sigma_k, P_4 = 1: (1 + s g_mu) psi = (h, s P_mu^dag h) with
// h = psi_up + s P_mu psi_low, so only two colour vectors meet the link.
#pragma once

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

// the forward (x + mu) hop of one direction for NR columns starting at col0
template <int P, int NE, bool DAG, int MU, int NR, typename R>
__device__ __forceinline__ void hop_fwd(const WilsonArgs& A, const int c[4], int par, int cb, int col0, int nv,
                                        cx<R> (*acc)[12]) {
  const Geom& g = A.g;
  const int pin = par ^ 1;
  cx<R> U[9];
  const int nb = nb_cb(c, MU, 1, g);
  load_link<P, NE>(A.links, g.Vh, par, MU, cb, U);
  const bool flip = (MU == 3 && g.ap && c[3] == g.L[3] - 1);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nv) {
      cx<R> psi[12], h[6], uh[6];
      IO<P, 12>::load(A.in, blk_index(A.in, col0 + r, pin), nb, psi);
      project<MU, DAG ? 1 : -1>(psi, h);
      if (flip) {
#pragma unroll
        for (int i = 0; i < 6; ++i) h[i] = -h[i];
      }
      if constexpr (P == 16) {
        su3_mv_chain(U, h, uh);
        su3_mv_chain(U, h + 3, uh + 3);
      } else {
        su3_mv(U, h, uh);
        su3_mv(U, h + 3, uh + 3);
      }
      recon_add<MU, DAG ? 1 : -1>(acc[r], uh);
    }
  }
}

// the backward (x - mu) hop
template <int P, int NE, bool DAG, int MU, int NR, typename R>
__device__ __forceinline__ void hop_bwd(const WilsonArgs& A, const int c[4], int par, int cb, int col0, int nv,
                                        cx<R> (*acc)[12]) {
  const Geom& g = A.g;
  const int pin = par ^ 1;
  cx<R> U[9];
  const int nb = nb_cb(c, MU, -1, g);
  load_link<P, NE>(A.links, g.Vh, pin, MU, nb, U);
  const bool flip = (MU == 3 && g.ap && c[3] == 0);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nv) {
      cx<R> psi[12], h[6], uh[6];
      IO<P, 12>::load(A.in, blk_index(A.in, col0 + r, pin), nb, psi);
      project<MU, DAG ? -1 : 1>(psi, h);
      if (flip) {
#pragma unroll
        for (int i = 0; i < 6; ++i) h[i] = -h[i];
      }
      if constexpr (P == 16) {
        su3_mv_dag_chain(U, h, uh);
        su3_mv_dag_chain(U, h + 3, uh + 3);
      } else {
        su3_mv_dag(U, h, uh);
        su3_mv_dag(U, h + 3, uh + 3);
      }
      recon_add<MU, DAG ? -1 : 1>(acc[r], uh);
    }
  }
}

// 6x6 complex matrix [36] (row-major) times the chiral half of a spinor
template <int P, typename R>
__device__ __forceinline__ void apply_full6(const void* base, int Vh, int par, int chir, int cb, const cx<R>* v,
                                            cx<R>* y) {
  using T2 = typename LinkT<P>::T2;
  const T2* p = (const T2*)base;
  const int g = par * 2 + chir;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    cx<R> s = {0, 0};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      T2 d = ldx<true>(p + tix(g, i * 6 + j, 36, cb, Vh));
      fma(s, cx<R>{(R)d.x, (R)d.y}, v[j]);
    }
    y[i] = s;
  }
}

// the same for NR columns, each matrix entry loaded once; in place on v[r][off..off+5]
template <int P, int NR, typename R>
__device__ __forceinline__ void apply_full6_nr(const void* base, int Vh, int par, int chir, int cb, int nv,
                                               cx<R> (*v)[12], int off) {
  using T2 = typename LinkT<P>::T2;
  const T2* p = (const T2*)base;
  const int g = par * 2 + chir;
  cx<R> y[NR][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int r = 0; r < NR; ++r) y[r][i] = {0, 0};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      T2 d = ldx<true>(p + tix(g, i * 6 + j, 36, cb, Vh));
      const cx<R> m = {(R)d.x, (R)d.y};
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nv) fma(y[r][i], m, v[r][off + j]);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 6; ++i) v[r][off + i] = y[r][i];
}

// Hermitian 6x6 packed as 3 T2 of diagonal pairs + 15 lower entries (i>j, row order)
template <int P, typename R>
__device__ __forceinline__ void apply_herm6(const void* base, int Vh, int par, int chir, int cb, const cx<R>* v,
                                            cx<R>* y) {
  using T2 = typename LinkT<P>::T2;
  const T2* p = (const T2*)base;
  const int g = par * 2 + chir;
  R d[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T2 e = ldx<true>(p + tix(g, k, 18, cb, Vh));
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
      T2 e = ldx<true>(p + tix(g, k, 18, cb, Vh));
      ++k;
      cx<R> l = {(R)e.x, (R)e.y};
      fma(y[i], l, v[j]);
      fmac(y[j], l, v[i]);
    }
  }
}

// Minimum waves per SIMD asked of the compiler for the FP64 / FP32 variants (the
// register-blocked ones use up to 256 VGPRs; 1 leaves the register budget
// at 256 and occupancy at 2 waves).
#ifndef LQ_MINW64
#define LQ_MINW64 1
#endif
#ifndef LQ_MINW32
#define LQ_MINW32 1
#endif
template <int P, int NE, bool DAG, int EPI, int NR>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, kStencilMaxThreads),
                               amdgpu_waves_per_eu(P == 64 ? LQ_MINW64 : P == 32 ? LQ_MINW32 : 1)))
wilson_kernel(WilsonArgs A) {
  using R = typename RealOf<P>::T;
  constexpr bool XMY = EPI == EPI_XMY_CLOVINV || EPI == EPI_XMY_RTS;
  constexpr bool RED = EPI == EPI_XMY_RTS;
  if (A.ncol <= 0) return;
  const int ngrp = (A.ncol + NR - 1) / NR;
  int par, cb, grp, c[4], tile = 0;
  const int status = stencil_site(A.g, A.par_out, A.slab, ngrp, A.sh, par, cb, grp, c, &tile);
  // lanes past the end of the last tile stay only to join the wave reductions
  if (status == 0 || (!RED && status != 1)) return;
  const bool live = status == 1;
  const int col0 = grp * NR;
  const int nv = min(NR, A.ncol - col0);  // <= 0 for waves without columns

  cx<R> acc[NR][12];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[r][i] = {0, 0};
  // Hop order: the backward hops from t down to x, then the forward hops from
  // x up to t.  A spinor that one wave reads as its +mu neighbour is read as
  // the -mu neighbour by a wave started later (its tile lies further along
  // the traversal); reading -mu early and +mu late brings the two reads
  // closer in time, most for t, whose neighbours are furthest apart, so more
  // of the second reads hit L2 (3% on the 12-column FP32 Schur stencils
  // against forward-backward per direction).
  hop_bwd<P, NE, DAG, 3, NR>(A, c, par, cb, col0, nv, acc);
  hop_bwd<P, NE, DAG, 2, NR>(A, c, par, cb, col0, nv, acc);
  hop_bwd<P, NE, DAG, 1, NR>(A, c, par, cb, col0, nv, acc);
  hop_bwd<P, NE, DAG, 0, NR>(A, c, par, cb, col0, nv, acc);
  hop_fwd<P, NE, DAG, 0, NR>(A, c, par, cb, col0, nv, acc);
  hop_fwd<P, NE, DAG, 1, NR>(A, c, par, cb, col0, nv, acc);
  hop_fwd<P, NE, DAG, 2, NR>(A, c, par, cb, col0, nv, acc);
  hop_fwd<P, NE, DAG, 3, NR>(A, c, par, cb, col0, nv, acc);

  const R k = (R)A.k_hop;
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[r][i] = k * acc[r][i];

  if constexpr (EPI == EPI_CLOVINV_XPAY) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nv) continue;
      cx<R> x[12];
      IO<P, 12>::template load<true>(A.x, blk_index(A.x, col0 + r, par), cb, x);
#pragma unroll
      for (int i = 0; i < 12; ++i) acc[r][i] = acc[r][i] + x[i];
    }
  }
  if constexpr (EPI == EPI_CLOVINV || XMY || EPI == EPI_CLOVINV_XPAY) {
    apply_full6_nr<P, NR>(A.clov_inv, A.g.Vh, par, 0, cb, nv, acc, 0);
    apply_full6_nr<P, NR>(A.clov_inv, A.g.Vh, par, 1, cb, nv, acc, 6);
  }
  double red[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r) red[r][0] = red[r][1] = red[r][2] = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nv) continue;
    const int col = col0 + r;
    cx<R> out[12];
    if constexpr (EPI == EPI_HOP || EPI == EPI_CLOVINV || EPI == EPI_CLOVINV_XPAY) {
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = acc[r][i];
    } else if constexpr (XMY) {
      cx<R> x[12];
      IO<P, 12>::template load<true>(A.x, blk_index(A.x, col, par), cb, x);
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = x[i] - acc[r][i];
      if (live) {
        if constexpr (RED) {
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            red[r][0] += (double)out[i].re * (double)x[i].re + (double)out[i].im * (double)x[i].im;
            red[r][1] += (double)out[i].re * (double)x[i].im - (double)out[i].im * (double)x[i].re;
            red[r][2] += (double)out[i].re * (double)out[i].re + (double)out[i].im * (double)out[i].im;
          }
        }
      }
    } else if constexpr (EPI == EPI_XPAY || EPI == EPI_XPAY_G5 || EPI == EPI_CHEB) {
      cx<R> x[12];
      IO<P, 12>::template load<true>(A.x, blk_index(A.x, col, par), cb, x);
      const R a = A.acol ? (R)A.acol[col] : (R)A.a;
#pragma unroll
      for (int i = 0; i < 12; ++i) out[i] = a * x[i] + acc[r][i];
      if constexpr (EPI != EPI_XPAY) {
#pragma unroll
        for (int i = 6; i < 12; ++i) out[i] = -out[i];
      }
      if constexpr (EPI == EPI_CHEB) {
        cx<R> v[12];
        const R s1 = (R)A.s1, ck = (R)A.ck, s2 = (R)A.s2;
        IO<P, 12>::template load<true>(A.v, blk_index(A.v, col, par), cb, v);
#pragma unroll
        for (int i = 0; i < 12; ++i) out[i] = s1 * out[i] + ck * v[i];
        IO<P, 12>::template load<true>(A.b1, blk_index(A.b1, col, par), cb, v);
#pragma unroll
        for (int i = 0; i < 12; ++i) out[i] = out[i] + s2 * v[i];
        IO<P, 12>::template load<true>(A.b2, blk_index(A.b2, col, par), cb, v);
#pragma unroll
        for (int i = 0; i < 12; ++i) out[i] = out[i] - v[i];
      }
    } else if constexpr (EPI == EPI_SITE) {
      cx<R> x[12];
      IO<P, 12>::template load<true>(A.x, blk_index(A.x, col, par), cb, x);
      apply_herm6<P>(A.clov, A.g.Vh, par, 0, cb, x, out);
      apply_herm6<P>(A.clov, A.g.Vh, par, 1, cb, x + 6, out + 6);
      const R mu = (R)A.mu_tw;
#pragma unroll
      for (int i = 0; i < 6; ++i) out[i] = out[i] + mu * times_i(x[i]) + acc[r][i];
#pragma unroll
      for (int i = 6; i < 12; ++i) out[i] = out[i] - mu * times_i(x[i]) + acc[r][i];
    }
    if (live) IO<P, 12>::template store<true>(A.out, blk_index(A.out, col, par), cb, out);
  }
  if constexpr (RED) {
    // wave butterfly (fixed order) and one partial per (column, 64-site tile)
    const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
    const int ntile = (nsite + 63) >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nv) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        for (int o = 32; o > 0; o >>= 1) red[r][k] += __shfl_xor(red[r][k], o);
      if ((threadIdx.x & 63) == 0) {
        double* p = A.red + ((int64_t)(col0 + r) * ntile + tile) * 4;
        p[0] = red[r][0];
        p[1] = red[r][1];
        p[2] = red[r][2];
        p[3] = 0.0;
      }
    }
  }
}

template <int P, int NE, bool DAG, int EPI, int NR>
inline void launch_one(const WilsonArgs& A, int bs, hipStream_t s) {
  (void)bs;
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  const StencilGrid G = stencil_grid(nsite, (A.ncol + NR - 1) / NR, A.tpb, A.xcd);
  WilsonArgs B = A;
  B.sh = G.sh;
  wilson_kernel<P, NE, DAG, EPI, NR><<<dim3(G.blocks), dim3(G.threads), 0, s>>>(B);
}

// epilogues with register-blocked variants (NR > 1)
constexpr bool epi_blocked(int epi) {
  return epi == EPI_CLOVINV || epi == EPI_XMY_CLOVINV || epi == EPI_XPAY || epi == EPI_XPAY_G5 || epi == EPI_CHEB ||
         epi == EPI_XMY_RTS || epi == EPI_SITE || epi == EPI_CLOVINV_XPAY;
}

template <int P, int NE, int EPI>
inline int launch_nr(const WilsonArgs& A, int nr, int bs, hipStream_t s) {
  if (A.dag) {
    if (nr != 1) return -1;
    launch_one<P, NE, true, EPI, 1>(A, bs, s);
    return 0;
  }
  if constexpr (epi_blocked(EPI)) {
    switch (nr) {
      case 1: launch_one<P, NE, false, EPI, 1>(A, bs, s); return 0;
      case 2: launch_one<P, NE, false, EPI, 2>(A, bs, s); return 0;
      case 3: launch_one<P, NE, false, EPI, 3>(A, bs, s); return 0;
      case 4: launch_one<P, NE, false, EPI, 4>(A, bs, s); return 0;
      case 6:
        if constexpr (P != 64) {
          launch_one<P, NE, false, EPI, 6>(A, bs, s);
          return 0;
        }
        return -1;
      default: return -1;
    }
  }
  if (nr != 1) return -1;
  launch_one<P, NE, false, EPI, 1>(A, bs, s);
  return 0;
}

template <int P, int NE>
inline int launch_epi(const WilsonArgs& A, int nr, int bs, hipStream_t s) {
  switch (A.epi) {
    case EPI_HOP: return launch_nr<P, NE, EPI_HOP>(A, nr, bs, s);
    case EPI_XPAY: return launch_nr<P, NE, EPI_XPAY>(A, nr, bs, s);
    case EPI_XPAY_G5: return launch_nr<P, NE, EPI_XPAY_G5>(A, nr, bs, s);
    case EPI_CHEB: return launch_nr<P, NE, EPI_CHEB>(A, nr, bs, s);
    default: break;
  }
  if constexpr (P != 16) {
    switch (A.epi) {
      case EPI_CLOVINV: return launch_nr<P, NE, EPI_CLOVINV>(A, nr, bs, s);
      case EPI_XMY_CLOVINV: return launch_nr<P, NE, EPI_XMY_CLOVINV>(A, nr, bs, s);
      case EPI_XMY_RTS: return launch_nr<P, NE, EPI_XMY_RTS>(A, nr, bs, s);
      case EPI_CLOVINV_XPAY: return launch_nr<P, NE, EPI_CLOVINV_XPAY>(A, nr, bs, s);
      case EPI_SITE: return launch_nr<P, NE, EPI_SITE>(A, nr, bs, s);
      default: break;
    }
  }
  return -1;
}

template <int P>
int launch_wilson_prec(const WilsonArgs& A, int nr, int bs, hipStream_t s) {
  if constexpr (P != 64) {
    if (A.recon) return launch_epi<P, 6>(A, nr, bs, s);
  }
  return launch_epi<P, 9>(A, nr, bs, s);
}

}  // namespace lq
