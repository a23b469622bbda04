// Device-side building blocks shared by every kernel of liblq:
// complex arithmetic, lattice geometry, and the even-odd SoA field layouts.
//
// Field layout in HBM (all precisions): a field is a sequence of "site blocks",
// one per (column, parity).  A block holds NC complex components per site
// (NC = 12 for Wilson spinors: spin*3 + colour; NC = 3 for staggered colour
// vectors) stored component-major, site-minor, so that consecutive lanes of a
// wave read consecutive sites (coalesced):
//   FP64: double2        [block][NC][Vh]
//   FP32: float4 (2 cx)  [block][NC/2][Vh]       (NC = 12)
//         float2         [block][NC][Vh]         (NC = 3)
//   FP16: 8 x half (4 cx)[block][NC/4][Vh] + float norm [block][Vh] (NC = 12)
//         half2          [block][NC][Vh]   + float norm [block][Vh] (NC = 3)
// FP16 values are stored divided by the site norm = max |re|,|im| over the
// site's components (round to nearest even); the norm itself is FP32.
// block = column * npar + (npar == 2 ? lattice parity : 0).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lq {

// ---------------------------------------------------------------- complex
template <typename R> struct cx { R re, im; };

template <typename R> __host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R> __host__ __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a += b * c ; a += conj(b) * c
template <typename R> __host__ __device__ __forceinline__ void fma(cx<R>& a, cx<R> b, cx<R> c) {
  a.re += b.re * c.re - b.im * c.im;
  a.im += b.re * c.im + b.im * c.re;
}
template <typename R> __host__ __device__ __forceinline__ void fmac(cx<R>& a, cx<R> b, cx<R> c) {
  a.re += b.re * c.re + b.im * c.im;
  a.im += b.re * c.im - b.im * c.re;
}
template <typename R> __host__ __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __host__ __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }

template <int P> struct RealOf { using T = float; };
template <> struct RealOf<64> { using T = double; };

// ---------------------------------------------------------------- geometry
// Extents L = (Lx, Ly, Lz, Lt), all even.  Checkerboard index of a site:
// cb = x/2 + Lx/2 * (y + Ly * (z + Lz * t)); parity = (x+y+z+t) & 1.
struct Geom {
  int L[4];
  int Lxh;
  int Vh;
  int ap;  // antiperiodic time for fermions
};

__device__ __forceinline__ void cb_coords(int cb, int par, const Geom& g, int c[4]) {
  int xh = cb % g.Lxh;
  int r = cb / g.Lxh;
  c[1] = r % g.L[1];
  r /= g.L[1];
  c[2] = r % g.L[2];
  c[3] = r / g.L[2];
  c[0] = 2 * xh + ((c[1] + c[2] + c[3] + par) & 1);
}

__device__ __forceinline__ int coords_cb(const int c[4], const Geom& g) {
  return (c[0] >> 1) + g.Lxh * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

// cb index of c + k*mu (periodic wrap), k in {-3,-1,1,3}
__device__ __forceinline__ int nb_cb(const int c[4], int mu, int k, const Geom& g) {
  int d[4] = {c[0], c[1], c[2], c[3]};
  int v = d[mu] + k;
  if (v >= g.L[mu]) v -= g.L[mu];
  if (v < 0) v += g.L[mu];
  d[mu] = v;
  return coords_cb(d, g);
}

// ---------------------------------------------------------------- fields
struct FieldRef {
  void* data;
  float* norm;  // FP16 only
  int npar;     // 1 or 2 parities stored per column
  int Vh;
};

__device__ __forceinline__ int64_t blk_index(const FieldRef& f, int col, int par) {
  return (int64_t)col * f.npar + (f.npar == 2 ? par : 0);
}

template <int P, int NC> struct IO;

template <int NC> struct IO<64, NC> {
  using R = double;
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const double2* p = (const double2*)f.data + blk * NC * (int64_t)f.Vh + cb;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double2 d = p[(int64_t)c * f.Vh];
      v[c] = {d.x, d.y};
    }
  }
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    double2* p = (double2*)f.data + blk * NC * (int64_t)f.Vh + cb;
#pragma unroll
    for (int c = 0; c < NC; ++c) p[(int64_t)c * f.Vh] = make_double2(v[c].re, v[c].im);
  }
};

template <> struct IO<32, 12> {
  using R = float;
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const float4* p = (const float4*)f.data + blk * 6 * (int64_t)f.Vh + cb;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 d = p[(int64_t)k * f.Vh];
      v[2 * k] = {d.x, d.y};
      v[2 * k + 1] = {d.z, d.w};
    }
  }
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    float4* p = (float4*)f.data + blk * 6 * (int64_t)f.Vh + cb;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      p[(int64_t)k * f.Vh] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
  }
};

template <> struct IO<32, 3> {
  using R = float;
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const float2* p = (const float2*)f.data + blk * 3 * (int64_t)f.Vh + cb;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 d = p[(int64_t)c * f.Vh];
      v[c] = {d.x, d.y};
    }
  }
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    float2* p = (float2*)f.data + blk * 3 * (int64_t)f.Vh + cb;
#pragma unroll
    for (int c = 0; c < 3; ++c) p[(int64_t)c * f.Vh] = make_float2(v[c].re, v[c].im);
  }
};

__device__ __forceinline__ float h2f(unsigned short h) { return __half2float(__ushort_as_half(h)); }
__device__ __forceinline__ unsigned short f2h(float f) { return __half_as_ushort(__float2half_rn(f)); }

template <int NC>
__device__ __forceinline__ float site_maxabs(const cx<float>* v) {
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
  return m;
}

template <> struct IO<16, 12> {
  using R = float;
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const uint4* p = (const uint4*)f.data + blk * 3 * (int64_t)f.Vh + cb;
    const float n = f.norm[blk * f.Vh + cb];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 d = p[(int64_t)k * f.Vh];
      unsigned w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[4 * k + j] = {n * h2f((unsigned short)(w[j] & 0xffffu)), n * h2f((unsigned short)(w[j] >> 16))};
    }
  }
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    uint4* p = (uint4*)f.data + blk * 3 * (int64_t)f.Vh + cb;
    const float n = site_maxabs<12>(v);
    const float s = n > 0.f ? 1.0f / n : 0.f;
    f.norm[blk * f.Vh + cb] = n;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      unsigned w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        w[j] = (unsigned)f2h(s * v[4 * k + j].re) | ((unsigned)f2h(s * v[4 * k + j].im) << 16);
      p[(int64_t)k * f.Vh] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
};

template <> struct IO<16, 3> {
  using R = float;
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const unsigned* p = (const unsigned*)f.data + blk * 3 * (int64_t)f.Vh + cb;
    const float n = f.norm[blk * f.Vh + cb];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      unsigned w = p[(int64_t)c * f.Vh];
      v[c] = {n * h2f((unsigned short)(w & 0xffffu)), n * h2f((unsigned short)(w >> 16))};
    }
  }
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    unsigned* p = (unsigned*)f.data + blk * 3 * (int64_t)f.Vh + cb;
    const float n = site_maxabs<3>(v);
    const float s = n > 0.f ? 1.0f / n : 0.f;
    f.norm[blk * f.Vh + cb] = n;
#pragma unroll
    for (int c = 0; c < 3; ++c) p[(int64_t)c * f.Vh] = (unsigned)f2h(s * v[c].re) | ((unsigned)f2h(s * v[c].im) << 16);
  }
};

// Bytes of one site of one block (without FP16 norms) and of the norm.
__host__ __device__ inline int site_bytes(int prec, int nc) { return prec == 64 ? nc * 16 : prec == 32 ? nc * 8 : nc * 4; }

// ---------------------------------------------------------------- links
// Link field layout: T2 elements [parity][mu][NE][Vh] with NE = 9 (full 3x3,
// row-major) or 6 (first two rows, third reconstructed as conj(row0 x row1)).
// FP16 links are unscaled for unitary fields; HISQ fields carry a per-field
// FP32 scale applied by the kernel.
template <int P> struct LinkT;
template <> struct LinkT<64> { using T2 = double2; };
template <> struct LinkT<32> { using T2 = float2; };
template <> struct LinkT<16> { using T2 = unsigned; };

template <int P, int NE>
__device__ __forceinline__ void load_link(const void* base, int Vh, int par, int mu, int cb,
                                          cx<typename RealOf<P>::T>* U) {
  using R = typename RealOf<P>::T;
  const int64_t off = ((int64_t)(par * 4 + mu) * NE) * Vh + cb;
  if constexpr (P == 64) {
    const double2* p = (const double2*)base + off;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      double2 d = p[(int64_t)e * Vh];
      U[e] = {d.x, d.y};
    }
  } else if constexpr (P == 32) {
    const float2* p = (const float2*)base + off;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      float2 d = p[(int64_t)e * Vh];
      U[e] = {d.x, d.y};
    }
  } else {
    const unsigned* p = (const unsigned*)base + off;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      unsigned w = p[(int64_t)e * Vh];
      U[e] = {h2f((unsigned short)(w & 0xffffu)), h2f((unsigned short)(w >> 16))};
    }
  }
  if constexpr (NE == 6) {
    U[6] = conj(U[1] * U[5] - U[2] * U[4]);
    U[7] = conj(U[2] * U[3] - U[0] * U[5]);
    U[8] = conj(U[0] * U[4] - U[1] * U[3]);
  }
  (void)sizeof(R);
}

// y = U x, y = U^dag x for colour vectors
template <typename R>
__device__ __forceinline__ void su3_mv(const cx<R>* U, const cx<R>* x, cx<R>* y) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = U[3 * a] * x[0];
    fma(s, U[3 * a + 1], x[1]);
    fma(s, U[3 * a + 2], x[2]);
    y[a] = s;
  }
}
template <typename R>
__device__ __forceinline__ void su3_mv_dag(const cx<R>* U, const cx<R>* x, cx<R>* y) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = cmulc(U[a], x[0]);
    fmac(s, U[3 + a], x[1]);
    fmac(s, U[6 + a], x[2]);
    y[a] = s;
  }
}

// XCD-aware block order: consecutive logical tiles go to the same XCD (the
// hardware dispatches workgroups round-robin over 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int nx = 8;
  if (nb < nx * 2) return b;
  const int per = nb / nx;          // full chunk per XCD
  const int rem_start = per * nx;   // blocks beyond go unmapped
  if (b >= rem_start) return b;
  return (b % nx) * per + b / nx;
}

}  // namespace lq
