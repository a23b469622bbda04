// Kernel launch descriptors and launchers of liblq (host-callable, defined in
// the .hip files).  Every launcher enqueues on the given stream and returns 0,
// or a negative status when the launch itself fails.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lq_common.h"

namespace lq {

// ------------------------------------------------------------ Wilson type
// EPI_XMY_RTS: EPI_XMY_CLOVINV plus the per-column reductions <out, x> and
// |out|^2 written as wave partials red[(col * ntile + tile) * 4 + k]
// (ntile = 64-site tiles of the launch).  EPI_CLOVINV_XPAY: A^{-1} (x + k hop)
// (the even-odd source and the odd-site reconstruction of the twisted clover).
enum { EPI_HOP = 0, EPI_XPAY, EPI_XPAY_G5, EPI_CLOVINV, EPI_XMY_CLOVINV, EPI_SITE, EPI_CHEB, EPI_XMY_RTS,
       EPI_CLOVINV_XPAY };

struct WilsonArgs {
  Geom g;
  int prec, recon, dag, epi;
  int par_out;  // 0, 1, or 2 = both parities
  int ncol;
  int slab;     // site traversal order code (0: lexicographic), see traversal_block
  int tpb, xcd; // site tiles per workgroup (0: automatic), XCD-aware block order
  int sh;       // packed launch shape, set by the launcher
  int nr;       // columns per thread (register blocking): 1, 2, 3, 4 or 6
  const void* links;
  FieldRef in, out, x, v, b1, b2;
  const void* clov;      // packed Hermitian H = (4+m) + C per chirality
  const void* clov_inv;  // full complex A^{-1} per chirality
  const double* acol;    // per-column coefficient of x (or nullptr: use a)
  double a, k_hop, mu_tw, s1, ck, s2;
  double* red;           // fused-reduction partials (EPI_XMY_RTS)
};
int launch_wilson(const WilsonArgs& A, hipStream_t s);
template <int P>
int launch_wilson_prec(const WilsonArgs& A, int nr, int bs, hipStream_t s);

// site term of the twisted-clover operator: out = A x or A^{-1} x per site
int launch_site(const Geom& g, int prec, const void* clov, const void* clov_inv, double mu_tw, bool inverse,
                FieldRef in, FieldRef out, int par_out, int ncol, hipStream_t s);

// ------------------------------------------------------------ staggered
// SEPI_XPAY_DOT: SEPI_XPAY plus the per-column <x, out> written as wave
// partials red[(col * ntile + tile) * 4 + {0: re, 1: im}] (ntile = 64-site
// tiles of the launch)
enum { SEPI_HOP = 0, SEPI_XPAY, SEPI_XPAY_DOT };

struct StagArgs {
  Geom g;
  int prec, epi, par_out, ncol;
  int slab;      // site traversal order code (0: lexicographic), see traversal_block
  int tpb, xcd;  // site tiles per workgroup (0: automatic), XCD-aware block order
  int sh;        // packed launch shape, set by the launcher
  int nr;  // columns per thread: 1, 2, 3, 4, 6 or 8
  const void* fat;
  const void* lng;
  float sfat, slong;
  FieldRef in, out, x;
  const double* acol;
  double a, k_hop;
  double* red;  // SEPI_XPAY_DOT partials
};
int launch_stag(const StagArgs& A, hipStream_t s);

// ------------------------------------------------------------ packing
// canonical AoS (device, FP64 complex): gauge [V][4][3][3]; spinor [col][V][NC]
int launch_pack_links(const Geom& g, const double* aos, void* out, int prec, int ne, int hisq_phases,
                      double scale, hipStream_t s);
int launch_pack_field(const Geom& g, const double* aos, int ncol, int nc, FieldRef out, int prec, int par_sel,
                      hipStream_t s);
int launch_unpack_field(const Geom& g, FieldRef in, int prec, int ncol, int nc, double* aos, int par_sel,
                        hipStream_t s);
int launch_convert(FieldRef dst, int pdst, FieldRef src, int psrc, int nc, int ncol, int npar, int Vh,
                   hipStream_t s);
double link_maxabs(const double* aos, int64_t n, hipStream_t s);

// ------------------------------------------------------------ clover (FP64 build)
int launch_clover_build(const Geom& g, const void* links64, double csw, double m, double mu, void* H64,
                        void* Ainv64, hipStream_t s);
int launch_clover_convert(const void* src64, void* dst32, int64_t n_t2, hipStream_t s);

// ------------------------------------------------------------ BLAS / reductions
enum {
  OP_AXPY = 0,   // f1 += c0 * f0
  OP_AXMY,       // f1 -= c0 * f0
  OP_XPAY,       // f1 = f0 + c0 * f1
  OP_CG,         // f2 += c0 f0 ; f3 -= c0 f1 ; red |f3|^2
  OP_BICG_XR,    // f3 += c0 f0 + c1 f1 ; f1 = f1 - c1 f2 ; red <f4,f1>, |f1|^2   (c0=alpha, c1=omega)
  OP_BICG_P,     // f2 = f0 + c0 (f2 - c1 f1)                                     (c0=beta, c1=omega)
  OP_DOT,        // red <f0, f1>
  OP_NORM2,      // red |f0|^2
  OP_DOT_NORM,   // red <f0, f1>, |f0|^2
  OP_XMY_NORM,   // f1 = f0 - f1 ; red |f1|^2
  OP_ZERO,       // f0 = 0
  OP_SCALE,      // f0 *= c0
  OP_G5,         // f1 = g5 f0 (Wilson only)
  OP_LC_G5,      // f2 = c0 f0 + c1 g5 f1 (Wilson only)
  OP_COPY,       // f1 = f0
  OP_PLC,        // f2 = p0 f0 + p1 (p2 f1 + p3 g5 f1), real p0..p3 per column from pcol (Wilson only)
  OP_NCOUNT
};

constexpr int ST_STRIDE = 16;  // doubles of solver state per column
// ST_NRST: CG direction restarts after a loss of positivity of <p, A p>
enum { ST_RHO = 0, ST_ALPHA = 2, ST_OMEGA = 4, ST_BETA = 6, ST_RR = 8, ST_FLAG = 9, ST_ACTIVE = 10, ST_AUX = 11,
       ST_RR0 = 13, ST_PAD = 14, ST_NRST = 15 };

struct BlasArgs {
  int prec, nc, ncol, npar, Vh, op;
  FieldRef f[5];
  const double* st;  // solver state [col][ST_STRIDE]; nullptr: use imm
  int c0, c1;        // offsets of complex coefficients in the state
  double imm[4];     // immediate coefficients c0 = imm[0] + i imm[1], c1 = imm[2] + i imm[3]
  double* partial;   // [ncol][gridx][4]
  int gridx;
  const double* pcol;  // OP_PLC: [ncol][4] real coefficients (device)
};
int launch_blas(const BlasArgs& A, hipStream_t s);
int blas_gridx(int64_t nsite);

// y(prec_y) += x(prec_x) element-wise, both with the same shape
int launch_axpy_mixed(FieldRef y, int py, FieldRef x, int px, int nc, int ncol, int npar, int Vh, hipStream_t s);

// scalar recurrences
enum { SC_CG_ALPHA = 0, SC_CG_BETA, SC_BICG_ALPHA, SC_BICG_OMEGA, SC_BICG_BETA, SC_SET_RR, SC_SET_RHO_RR,
       SC_DOT_TO_AUX };
int launch_scalar(int op, const double* partial, int gridx, int ncol, double* st, hipStream_t s);

// multi-shift CG (Jegerlehner): fields with ncol = nshift * nrhs, shift-major
struct MsArgs {
  int prec, nc, nrhs, nshift, npar, Vh;
  FieldRef x, p, r, ap;
  double* sh;  // shift state [nshift][nrhs][8]
  double* st;  // base state [nrhs][ST_STRIDE]
  double* partial;
  int gridx;
};
int launch_ms_xr(const MsArgs& A, hipStream_t s);     // r -= a Ap ; red |r|^2
int launch_ms_p(const MsArgs& A, hipStream_t s);      // x_i += a_i p_i ; p_i = z_i r + b_i p_i (p_0: z = 1)
int launch_ms_scalar_alpha(const MsArgs& A, const double* sigma, hipStream_t s);
int launch_ms_scalar_beta(const MsArgs& A, hipStream_t s);
int launch_ms_init(const MsArgs& A, hipStream_t s);

// ------------------------------------------------------------ multigrid
// Two-level aggregation: Vc aggregates of B fine sites, nv near-null vectors
// (2 nv <= 64 and a multiple of 12); coarse vectors are Wilson-shaped fields of
// K = 2 nv / 12 pseudo-sites per aggregate (npar = 1, Vh = K Vc).  Basis
// Q[Vc][B][2][nv][6], coarse operator Dc[Vc][9][2nv][2nv] (see mg.hip).
struct MgGeom {
  int Vc, B, nv, K;
  const int* fine;   // [Vc * B]: fine site cb | parity << 30 of (aggregate, in-block index)
  const int* nbr;    // [Vc][8]: aggregate at Y + mu (2 mu) and Y - mu (2 mu + 1)
  const int* face;   // [Vc * B]: bit 2 mu: lowest layer in mu, bit 2 mu + 1: highest layer
  const int* cpar;   // [Vc]: coarse coordinate parities, bit mu = Y_mu & 1
  const int* cmap;   // [Vc]: coarse checkerboard index | coarse parity << 30
  const int* csite;  // [2][Vc / 2]: aggregate of (parity, checkerboard index)
};
int launch_mg_restrict(const MgGeom& m, int pf, const void* Q, FieldRef fine, int pc, FieldRef coarse, int ncol,
                       hipStream_t s);
int launch_mg_prolong(const MgGeom& m, int pc, FieldRef coarse, int pf, const void* Q, FieldRef fine, int ncol,
                      hipStream_t s);
// out(Y) = a x(Y) + sgn sum_{d0 <= d < d0 + nd} M[Y][d] in(N_d(Y)) on the aggregates of parity par_out (2: all)
int launch_mg_stencil(const MgGeom& m, int p, const void* M, int d0, int nd, FieldRef in, FieldRef out, FieldRef x,
                      double a, double sgn, int par_out, int ncol, hipStream_t s);
// Ahat[Y][0] = Dc[Y][0]^{-1} (FP64; work: Vc * 2 (2 nv)^2 complex), then Ahat[Y][d] = Ahat[Y][0] Dc[Y][d], d = 1..8
int launch_mg_site_inverse(const MgGeom& m, const void* Dc64, void* Ahat64, void* work, int* bad, hipStream_t s);
int launch_mg_site_mul(const MgGeom& m, const void* Dc64, void* Ahat64, hipStream_t s);
int launch_mg_gather(const MgGeom& m, FieldRef fine, void* Q64, hipStream_t s);
int launch_mg_orth(const MgGeom& m, void* Q64, int* bad, hipStream_t s);
int launch_mg_probe_restrict(const MgGeom& m, const void* Q64, FieldRef fine, int ncol, int k0, int cls, void* Dc64,
                             hipStream_t s);
int launch_mg_narrow(const void* src64, void* dst32, int64_t n_complex, hipStream_t s);
int launch_mg_random(FieldRef fine, int ncol, uint64_t seed, hipStream_t s);

// profiling-free utilities
int launch_fill_zero(void* p, size_t bytes, hipStream_t s);
int launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// exchange two non-overlapping byte ranges of equal length (16-byte aligned)
int launch_swap_bytes(void* a, void* b, size_t bytes, hipStream_t s);

}  // namespace lq
