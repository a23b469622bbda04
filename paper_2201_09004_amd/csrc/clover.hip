// Clover (Sheikholeslami-Wohlert) term and twisted-mass site inverse, built
// on the device in FP64 (sec. 2.1, eq. 3; the twisted inverse has a complex
// diagonal and cannot use the Hermitian packing, so it is computed here).
//
// Convention (Luescher normalisation):
//   C(x) = -(c_sw/2) sum_{mu<nu} g_mu g_nu (x) F_{mu nu}(x),
//   F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/8 made traceless,
// Q the sum of the four plaquette leaves around x.  In the chiral basis
// g_mu g_nu is block diagonal; with G_x = F_yz, G_y = -F_xz, G_z = F_xy,
// E_k = F_kt and X^{+-}_k = i (G_k -+ E_k) (Hermitian 3x3),
//   C_{+-} = -(c_sw/2) [[X_z, X_x - i X_y], [X_x + i X_y, -X_z]]   (6x6).
// H_{+-} = (4+m) + C_{+-} is stored packed Hermitian; the site term of the
// twisted operator is A_{+-} = H_{+-} +- i mu and its inverse is stored as a
// full complex 6x6 per chirality (Gauss-Jordan with partial pivoting).
#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

using C = cx<double>;

struct M3 { C e[9]; };

__device__ __forceinline__ M3 mm(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C s = a.e[3 * i] * b.e[j];
      fma(s, a.e[3 * i + 1], b.e[3 + j]);
      fma(s, a.e[3 * i + 2], b.e[6 + j]);
      r.e[3 * i + j] = s;
    }
  return r;
}
__device__ __forceinline__ M3 dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 * i + j] = conj(a.e[3 * j + i]);
  return r;
}

__device__ __forceinline__ M3 link_at(const void* links, const Geom& g, const int c[4], int mu) {
  const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
  M3 u;
  load_link<64, 9>(links, g.Vh, par, mu, coords_cb(c, g), u.e);
  return u;
}

__device__ __forceinline__ void step(int c[4], int mu, int k, const Geom& g) {
  int v = c[mu] + k;
  if (v >= g.L[mu]) v -= g.L[mu];
  if (v < 0) v += g.L[mu];
  c[mu] = v;
}

// Q_{mu nu}(x): four counter-clockwise leaves, each walked link by link
__device__ M3 leaves(const void* links, const Geom& g, const int x[4], int mu, int nu) {
  M3 q;
#pragma unroll
  for (int i = 0; i < 9; ++i) q.e[i] = {0, 0};
  const int path[4][4][2] = {{{mu, 1}, {nu, 1}, {mu, -1}, {nu, -1}},
                             {{nu, 1}, {mu, -1}, {nu, -1}, {mu, 1}},
                             {{mu, -1}, {nu, -1}, {mu, 1}, {nu, 1}},
                             {{nu, -1}, {mu, 1}, {nu, 1}, {mu, -1}}};
  for (int l = 0; l < 4; ++l) {
    int c[4] = {x[0], x[1], x[2], x[3]};
    M3 prod;
    for (int i = 0; i < 9; ++i) prod.e[i] = {(i % 4 == 0) ? 1.0 : 0.0, 0.0};
    for (int s = 0; s < 4; ++s) {
      const int d = path[l][s][0], f = path[l][s][1];
      if (f > 0) {
        prod = mm(prod, link_at(links, g, c, d));
        step(c, d, 1, g);
      } else {
        step(c, d, -1, g);
        prod = mm(prod, dag(link_at(links, g, c, d)));
      }
    }
    for (int i = 0; i < 9; ++i) q.e[i] = q.e[i] + prod.e[i];
  }
  return q;
}

__device__ M3 fstrength(const void* links, const Geom& g, const int x[4], int mu, int nu) {
  M3 q = leaves(links, g, x, mu, nu);
  M3 f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) f.e[3 * i + j] = 0.125 * (q.e[3 * i + j] - conj(q.e[3 * j + i]));
  C tr = (1.0 / 3.0) * (f.e[0] + f.e[4] + f.e[8]);
  f.e[0] = f.e[0] - tr;
  f.e[4] = f.e[4] - tr;
  f.e[8] = f.e[8] - tr;
  return f;
}

// in-place inverse of a 6x6 complex matrix (row-major), partial pivoting
__device__ void inv6(C* a, C* inv) {
  for (int i = 0; i < 36; ++i) inv[i] = {(i % 7 == 0) ? 1.0 : 0.0, 0.0};
  for (int k = 0; k < 6; ++k) {
    int piv = k;
    double best = a[6 * k + k].re * a[6 * k + k].re + a[6 * k + k].im * a[6 * k + k].im;
    for (int r = k + 1; r < 6; ++r) {
      double v = a[6 * r + k].re * a[6 * r + k].re + a[6 * r + k].im * a[6 * r + k].im;
      if (v > best) { best = v; piv = r; }
    }
    if (piv != k)
      for (int j = 0; j < 6; ++j) {
        C t = a[6 * k + j]; a[6 * k + j] = a[6 * piv + j]; a[6 * piv + j] = t;
        t = inv[6 * k + j]; inv[6 * k + j] = inv[6 * piv + j]; inv[6 * piv + j] = t;
      }
    const C p = a[6 * k + k];
    const double d = p.re * p.re + p.im * p.im;
    const C pinv = {p.re / d, -p.im / d};
    for (int j = 0; j < 6; ++j) { a[6 * k + j] = pinv * a[6 * k + j]; inv[6 * k + j] = pinv * inv[6 * k + j]; }
    for (int r = 0; r < 6; ++r) {
      if (r == k) continue;
      const C f = a[6 * r + k];
      for (int j = 0; j < 6; ++j) {
        a[6 * r + j] = a[6 * r + j] - f * a[6 * k + j];
        inv[6 * r + j] = inv[6 * r + j] - f * inv[6 * k + j];
      }
    }
  }
}

__global__ void clover_build_kernel(Geom g, const void* links, double csw, double m, double mu_tw, double2* H,
                                    double2* Ainv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * (int64_t)g.Vh) return;
  const int par = (int)(i / g.Vh);
  const int cb = (int)(i % g.Vh);
  int x[4];
  cb_coords(cb, par, g, x);
  M3 F01 = fstrength(links, g, x, 0, 1), F02 = fstrength(links, g, x, 0, 2), F12 = fstrength(links, g, x, 1, 2);
  M3 F03 = fstrength(links, g, x, 0, 3), F13 = fstrength(links, g, x, 1, 3), F23 = fstrength(links, g, x, 2, 3);
  const C I = {0, 1};
  for (int chir = 0; chir < 2; ++chir) {
    const double sg = chir == 0 ? -1.0 : 1.0;  // X = i (G - E) upper, i (G + E) lower
    C X[3][9];
    for (int e = 0; e < 9; ++e) {
      X[0][e] = I * (F12.e[e] + sg * F03.e[e]);
      X[1][e] = I * ((-1.0) * F02.e[e] + sg * F13.e[e]);
      X[2][e] = I * (F01.e[e] + sg * F23.e[e]);
    }
    C h[36];
    const double k = -0.5 * csw;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int e = 3 * a + b;
        h[6 * a + b] = k * X[2][e];
        h[6 * a + 3 + b] = k * (X[0][e] - I * X[1][e]);
        h[6 * (3 + a) + b] = k * (X[0][e] + I * X[1][e]);
        h[6 * (3 + a) + 3 + b] = (-k) * X[2][e];
      }
    for (int d = 0; d < 6; ++d) h[7 * d] = h[7 * d] + C{4.0 + m, 0.0};
    // packed Hermitian store: diag pairs then lower triangle in row order
    const int grp = par * 2 + chir;
    for (int kk = 0; kk < 3; ++kk)
      H[tix(grp, kk, 18, cb, g.Vh)] = make_double2(h[7 * (2 * kk)].re, h[7 * (2 * kk + 1)].re);
    int kk = 3;
    for (int r = 1; r < 6; ++r)
      for (int cc = 0; cc < r; ++cc) {
        H[tix(grp, kk, 18, cb, g.Vh)] = make_double2(h[6 * r + cc].re, h[6 * r + cc].im);
        ++kk;
      }
    // A = H +- i mu (g5 = +1 on the upper chirality)
    const double tw = chir == 0 ? mu_tw : -mu_tw;
    for (int d = 0; d < 6; ++d) h[7 * d] = h[7 * d] + C{0.0, tw};
    C inv[36];
    inv6(h, inv);
    for (int e = 0; e < 36; ++e) Ainv[tix(grp, e, 36, cb, g.Vh)] = make_double2(inv[e].re, inv[e].im);
  }
}

int launch_clover_build(const Geom& g, const void* links64, double csw, double m, double mu, void* H64, void* Ainv64,
                        hipStream_t s) {
  const int64_t n = 2 * (int64_t)g.Vh;
  const int bs = 64;
  clover_build_kernel<<<(int)((n + bs - 1) / bs), bs, 0, s>>>(g, links64, csw, m, mu, (double2*)H64,
                                                              (double2*)Ainv64);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

__global__ void t2_convert_kernel(const double2* src, float2* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

int launch_clover_convert(const void* src64, void* dst32, int64_t n_t2, hipStream_t s) {
  const int bs = 256;
  t2_convert_kernel<<<(int)((n_t2 + bs - 1) / bs), bs, 0, s>>>((const double2*)src64, (float2*)dst32, n_t2);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq
