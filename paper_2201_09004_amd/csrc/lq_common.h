// Device-side building blocks shared by every kernel of liblq:
// complex arithmetic, lattice geometry, and the even-odd field layouts.
//
// Field layout in HBM (all precisions): a field is a sequence of "site blocks",
// one per (column, parity).  A block holds the site data of Vh checkerboard
// sites as K chunks per site (a chunk is the unit one lane loads: 16 B for
// FP64 complex, FP32 complex pairs and FP16 complex quads; 8 B / 4 B for the
// staggered FP32 / FP16 colour components).  Chunks are stored in tiles of
// LQ_TILE consecutive sites: [block][Vh / LQ_TILE][K][LQ_TILE] (LQ_TILE = 1
// gives the plain component-plane layout [block][K][Vh]).  A wave of 64
// consecutive sites then reads whole cache lines for every chunk, and all of
// a site's data sits within a few kilobytes (few DRAM pages and TLB entries):
//   FP64: double2        K = NC
//   FP32: float4 (2 cx)  K = NC/2  (NC = 12)   float2  K = NC (NC = 3)
//   FP16: 8 x half (4 cx) K = NC/4 (NC = 12)   half2   K = NC (NC = 3)
//         + float norm [block][Vh]
// FP16 values are stored divided by the site norm = max |re|,|im| over the
// site's components (round to nearest even); the norm itself is FP32.
// block = column * npar + (npar == 2 ? lattice parity : 0).
// Links and site matrices use the same tiled map with K = elements per site.
// Vh is a multiple of 8 for even extents, so LQ_TILE = 8 always divides it.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lq {

// ---------------------------------------------------------------- complex
template <typename R> struct cx { R re, im; };

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
// real fused multiply-add, one rounding (v_fma_f32 / v_fma_f64)
__host__ __device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a += b c and a += conj(b) c as chains of four fused multiply-adds into a.
// Written as a + (x - y), as fma and fmac are, each real part costs a multiply,
// an FMA and an add; the chains take 4 instead of 6 instructions per complex
// multiply-add.  The FP16 Wilson stencils use them (their operands are
// converted inside the FMA, v_fma_mix_f32, and instruction issue bounds the
// kernel); the FP32 and FP64 stencils keep fma / fmac, with which the compiler's
// register allocation and occupancy measured faster.
template <typename R> __host__ __device__ __forceinline__ void cmadd(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fmar(b.re, c.re, a.re);
  a.re = fmar(-b.im, c.im, a.re);
  a.im = fmar(b.re, c.im, a.im);
  a.im = fmar(b.im, c.re, a.im);
}
template <typename R> __host__ __device__ __forceinline__ void cmadd_conj(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fmar(b.re, c.re, a.re);
  a.re = fmar(b.im, c.im, a.re);
  a.im = fmar(b.re, c.im, a.im);
  a.im = fmar(-b.im, c.re, a.im);
}
// FP16 operands packed as (re, im) pairs of halves: dot2h(a, b, c) = a.re b.re +
// a.im b.im + c in FP32 by v_dot2_f32_f16 (the product of two FP16 numbers is
// exact in FP32), so with m = (m.re, m.im) one real part of m x is one
// instruction: Re(m x) = dot2h((m.re, -m.im), x), Im(m x) = dot2h((m.im, m.re), x).
typedef _Float16 half2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2h(unsigned a, unsigned b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_v, a), __builtin_bit_cast(half2_v, b), c, false);
}
__device__ __forceinline__ unsigned swap_halves(unsigned w) { return (w >> 16) | (w << 16); }
// sign bits of the upper (im) and the lower (re) half
constexpr unsigned kSignHi = 0x80000000u, kSignLo = 0x00008000u;
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
#ifndef LQ_TILE
#define LQ_TILE 8
#endif

// element index of chunk k (of K per site) of site cb in group g of Vh sites
__host__ __device__ __forceinline__ int64_t tix(int64_t g, int k, int K, int cb, int Vh) {
#if LQ_TILE > 1
  return g * (int64_t)K * Vh + (int64_t)(cb / LQ_TILE) * (K * LQ_TILE) + k * LQ_TILE + (cb % LQ_TILE);
#else
  return (g * (int64_t)K + k) * Vh + cb;
#endif
}

// ---------------------------------------------------------------- streaming access
// Data that a stencil launch touches exactly once (links, site matrices, the
// output site's own operands and its result) goes through ldx/stx<true>.
// LQ_NT selects which of them carry the non-temporal hint, meant to leave L2
// to the neighbour spinors (each read by eight sites).  On gfx950 hinted loads
// made the stencils 20-30% slower, hinted stores 2-3% faster, so by default
// only the stores are hinted.
#ifndef LQ_NT
#define LQ_NT 2  // bit 0: streaming loads, bit 1: streaming stores
#endif
template <bool NT, typename T>
__device__ __forceinline__ T ldx(const T* p) {
  if constexpr (NT && (LQ_NT & 1) && (sizeof(T) == 16 || sizeof(T) == 8 || sizeof(T) == 4)) {
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    T out;
    if constexpr (sizeof(T) == 16) {
      const v4u r = __builtin_nontemporal_load((const v4u*)p);
      __builtin_memcpy(&out, &r, 16);
    } else if constexpr (sizeof(T) == 8) {
      const v2u r = __builtin_nontemporal_load((const v2u*)p);
      __builtin_memcpy(&out, &r, 8);
    } else {
      const unsigned r = __builtin_nontemporal_load((const unsigned*)p);
      __builtin_memcpy(&out, &r, 4);
    }
    return out;
  } else {
    return *p;
  }
}
template <bool NT, typename T>
__device__ __forceinline__ void stx(T* p, const T& v) {
  if constexpr (NT && (LQ_NT & 2) && (sizeof(T) == 16 || sizeof(T) == 8 || sizeof(T) == 4)) {
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 16) {
      v4u r;
      __builtin_memcpy(&r, &v, 16);
      __builtin_nontemporal_store(r, (v4u*)p);
    } else if constexpr (sizeof(T) == 8) {
      v2u r;
      __builtin_memcpy(&r, &v, 8);
      __builtin_nontemporal_store(r, (v2u*)p);
    } else {
      unsigned r;
      __builtin_memcpy(&r, &v, 4);
      __builtin_nontemporal_store(r, (unsigned*)p);
    }
  } else {
    *p = v;
  }
}

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
  template <bool NT = false>
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const double2* p = (const double2*)f.data;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double2 d = ldx<NT>(p + tix(blk, c, NC, cb, f.Vh));
      v[c] = {d.x, d.y};
    }
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    double2* p = (double2*)f.data;
#pragma unroll
    for (int c = 0; c < NC; ++c) stx<NT>(p + tix(blk, c, NC, cb, f.Vh), make_double2(v[c].re, v[c].im));
  }
};

template <> struct IO<32, 12> {
  using R = float;
  template <bool NT = false>
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const float4* p = (const float4*)f.data;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 d = ldx<NT>(p + tix(blk, k, 6, cb, f.Vh));
      v[2 * k] = {d.x, d.y};
      v[2 * k + 1] = {d.z, d.w};
    }
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    float4* p = (float4*)f.data;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      stx<NT>(p + tix(blk, k, 6, cb, f.Vh), make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im));
  }
};

template <> struct IO<32, 3> {
  using R = float;
  template <bool NT = false>
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const float2* p = (const float2*)f.data;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 d = ldx<NT>(p + tix(blk, c, 3, cb, f.Vh));
      v[c] = {d.x, d.y};
    }
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    float2* p = (float2*)f.data;
#pragma unroll
    for (int c = 0; c < 3; ++c) stx<NT>(p + tix(blk, c, 3, cb, f.Vh), make_float2(v[c].re, v[c].im));
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

// Site norm as stored for FP16: a site whose largest component is below the
// smallest normal FP32 number is stored as zero, because 1/n would overflow
// to infinity (and infinity times a zero component is NaN).  Such sites are
// at least 2^-126 times smaller than any normal site of the field.
__device__ __forceinline__ float fp16_site_norm(float n) { return n >= 1.17549435e-38f ? n : 0.f; }

template <> struct IO<16, 12> {
  using R = float;
  template <bool NT = false>
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const uint4* p = (const uint4*)f.data;
    const float n = ldx<NT>(f.norm + blk * f.Vh + cb);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 d = ldx<NT>(p + tix(blk, k, 3, cb, f.Vh));
      unsigned w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[4 * k + j] = {n * h2f((unsigned short)(w[j] & 0xffffu)), n * h2f((unsigned short)(w[j] >> 16))};
    }
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    uint4* p = (uint4*)f.data;
    const float n = fp16_site_norm(site_maxabs<12>(v));
    const float s = n > 0.f ? 1.0f / n : 0.f;
    stx<NT>(f.norm + blk * f.Vh + cb, n);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      unsigned w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        w[j] = (unsigned)f2h(s * v[4 * k + j].re) | ((unsigned)f2h(s * v[4 * k + j].im) << 16);
      stx<NT>(p + tix(blk, k, 3, cb, f.Vh), make_uint4(w[0], w[1], w[2], w[3]));
    }
  }
};

// FP16 staggered sites are packed with their norm in one 16-byte chunk
// (3 half2 + the FP32 norm), so a neighbour gather is one load
template <> struct IO<16, 3> {
  using R = float;
  template <bool NT = false>
  static __device__ __forceinline__ void load(const FieldRef& f, int64_t blk, int cb, cx<R>* v) {
    const uint4 d = ldx<NT>((const uint4*)f.data + tix(blk, 0, 1, cb, f.Vh));
    const float n = __uint_as_float(d.w);
    const unsigned w[3] = {d.x, d.y, d.z};
#pragma unroll
    for (int c = 0; c < 3; ++c)
      v[c] = {n * h2f((unsigned short)(w[c] & 0xffffu)), n * h2f((unsigned short)(w[c] >> 16))};
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(const FieldRef& f, int64_t blk, int cb, const cx<R>* v) {
    const float n = fp16_site_norm(site_maxabs<3>(v));
    const float s = n > 0.f ? 1.0f / n : 0.f;
    unsigned w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = (unsigned)f2h(s * v[c].re) | ((unsigned)f2h(s * v[c].im) << 16);
    stx<NT>((uint4*)f.data + tix(blk, 0, 1, cb, f.Vh), make_uint4(w[0], w[1], w[2], __float_as_uint(n)));
  }
};

// Bytes of one site of one block in the main array (FP16 Wilson-type sites
// keep their norm in a separate array, FP16 staggered sites hold it inline),
// and whether the precision and shape keep a separate norm array.
__host__ __device__ inline int site_bytes(int prec, int nc) {
  return prec == 64 ? nc * 16 : prec == 32 ? nc * 8 : (nc == 3 ? 16 : nc * 4);
}
__host__ __device__ inline bool sep_norm(int prec, int nc) { return prec == 16 && nc != 3; }

// ---------------------------------------------------------------- links
// Link fields: T2 elements in groups (parity, mu) of NE elements per site
// (NE = 9: full 3x3 row-major; NE = 6: first two rows, the third rebuilt as
// conj(row0 x row1)), tiled as the fields above.  FP16 links are unscaled for
// unitary fields; HISQ fields carry a per-field FP32 scale applied by the kernel.
template <int P> struct LinkT;
template <> struct LinkT<64> { using T2 = double2; };
template <> struct LinkT<32> { using T2 = float2; };
template <> struct LinkT<16> { using T2 = unsigned; };

template <int P, int NE>
__device__ __forceinline__ void load_link(const void* base, int Vh, int par, int mu, int cb,
                                          cx<typename RealOf<P>::T>* U) {
  const int g = par * 4 + mu;
  if constexpr (P == 64) {
    const double2* p = (const double2*)base;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      double2 d = ldx<true>(p + tix(g, e, NE, cb, Vh));
      U[e] = {d.x, d.y};
    }
  } else if constexpr (P == 32) {
    const float2* p = (const float2*)base;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      float2 d = ldx<true>(p + tix(g, e, NE, cb, Vh));
      U[e] = {d.x, d.y};
    }
  } else {
    const unsigned* p = (const unsigned*)base;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      unsigned w = ldx<true>(p + tix(g, e, NE, cb, Vh));
      U[e] = {h2f((unsigned short)(w & 0xffffu)), h2f((unsigned short)(w >> 16))};
    }
  }
  if constexpr (NE == 6) {
    U[6] = conj(U[1] * U[5] - U[2] * U[4]);
    U[7] = conj(U[2] * U[3] - U[0] * U[5]);
    U[8] = conj(U[0] * U[4] - U[1] * U[3]);
  }
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
// the same with fused multiply-add chains (FP16 Wilson stencils)
template <typename R>
__device__ __forceinline__ void su3_mv_chain(const cx<R>* U, const cx<R>* x, cx<R>* y) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = U[3 * a] * x[0];
    cmadd(s, U[3 * a + 1], x[1]);
    cmadd(s, U[3 * a + 2], x[2]);
    y[a] = s;
  }
}
template <typename R>
__device__ __forceinline__ void su3_mv_dag_chain(const cx<R>* U, const cx<R>* x, cx<R>* y) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = cmulc(U[a], x[0]);
    cmadd_conj(s, U[3 + a], x[1]);
    cmadd_conj(s, U[6 + a], x[2]);
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

// Site traversal order of the stencil kernels.  The lattice of one parity is
// cut into blocks of by x bz x bt (y, z, t) planes holding whole x rows; the
// blocks are walked with y fastest, then z, then t, and each block is walked
// lexicographically (x, y, z, t) inside.  A block small enough that the sites
// in flight on one XCD cover most of it keeps the neighbour spinors of all
// eight directions in that XCD's L2.  The code is the tuned knob:
//   0         lexicographic (one block: by = Ly, bz = Lz, bt = Lt)
//   1 .. 255  slabs of that many z planes (by = Ly, bt = Lt)
//   otherwise by | bz << 8 | bt << 16
__host__ __device__ inline void traversal_block(const Geom& g, int code, int& by, int& bz, int& bt) {
  if (code <= 0) {
    by = g.L[1], bz = g.L[2], bt = g.L[3];
  } else if (code < 256) {
    by = g.L[1], bz = code, bt = g.L[3];
  } else {
    by = code & 0xff, bz = (code >> 8) & 0xff, bt = (code >> 16) & 0xff;
  }
}
inline bool traversal_valid(const Geom& g, int code) {
  if (code < 0) return false;
  int by, bz, bt;
  traversal_block(g, code, by, bz, bt);
  return by > 0 && bz > 0 && bt > 0 && g.L[1] % by == 0 && g.L[2] % bz == 0 && g.L[3] % bt == 0;
}
inline int traversal_code(int by, int bz, int bt) { return by | (bz << 8) | (bt << 16); }

// Work decomposition of the stencil kernels.  A workgroup owns one tile of 64
// consecutive sites (in traversal order) and gw = blockDim.x / 64 column
// groups, one wave per group, so every column group of a site runs on the same
// CU and the links and site matrices of the tile are fetched from HBM once.
// Sites are taken in the traversal order given by the code (see
// traversal_block).
// Launch shape knobs (tuned): sh = gw | tpb << 8 | xcd << 16 with gw column
// groups and tpb site tiles per workgroup (one wave each), xcd = 1 to apply
// xcd_remap to the block index.
// Returns 0 when the whole wave has no sites (it can exit), 1 for a lane with
// a site, 2 for a lane of the last, partial tile past the end (its site is
// clamped to the last one so that it can still join wave-wide reductions).
__device__ __forceinline__ int stencil_site(const Geom& g, int par_out, int order, int ngrp, int sh, int& par,
                                            int& cb, int& grp, int c[4], int* tile_out = nullptr) {
  const int nsite = par_out == 2 ? 2 * g.Vh : g.Vh;
  const int ntile = (nsite + 63) >> 6;
  const int gw = sh & 0xff, tpb = (sh >> 8) & 0xff;
  const int nchunk = (ngrp + gw - 1) / gw;
  const int lb = ((sh >> 16) & 1) ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int bt = lb / nchunk;
  // the wave index is uniform across the wave: keep it (and the column group
  // and field base addresses derived from it) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = bt * tpb + w / gw;
  grp = (lb - bt * nchunk) * gw + (w % gw);
  int j = tile * 64 + (threadIdx.x & 63);
  // Waves past the last column group (grp >= ngrp, when gw does not divide
  // ngrp) are not turned away here: the kernels give them no columns
  // (ncol - grp*NR <= 0), so they only read valid addresses and store
  // nothing.  An explicit grp check lets the compiler prove every column
  // guard true and merge the whole stencil into one block, which doubles
  // register use and spills.
  (void)ngrp;
  if (tile >= ntile) return 0;
  if (tile_out) *tile_out = tile;
  const int status = j < nsite ? 1 : 2;
  if (j >= nsite) j = nsite - 1;
  par = par_out == 2 ? (j >= g.Vh ? 1 : 0) : par_out;
  const int jj = par_out == 2 ? j - par * g.Vh : j;
  int oy, oz, ot;  // traversal block extents
  traversal_block(g, order, oy, oz, ot);
  const int xh = jj % g.Lxh;
  const int r = jj / g.Lxh;  // x row in traversal order
  const int rows = oy * oz * ot;
  const int blk = r / rows;
  int q = r - blk * rows;
  const int yi = q % oy;
  q /= oy;
  const int zi = q % oz;
  const int ti = q / oz;
  const int nby = g.L[1] / oy, nbz = g.L[2] / oz;
  const int yb = blk % nby, b2 = blk / nby;
  // coordinates as scalars, each stored once (stores in alternative branches
  // would be merged into one store through a selected pointer, which keeps
  // the coordinate array in scratch memory)
  const int y = yb * oy + yi, z = (b2 % nbz) * oz + zi, t = (b2 / nbz) * ot + ti;
  c[1] = y;
  c[2] = z;
  c[3] = t;
  c[0] = 2 * xh + ((y + z + t + par) & 1);
  cb = xh + g.Lxh * (y + g.L[1] * (z + g.L[2] * t));
  return status;
}

// launch shape matching stencil_site: 64 sites x gw groups per workgroup, at
// most 4 waves (256-thread launch bounds leave the register-blocked variants
// up to 256 VGPRs)
constexpr int kStencilMaxThreads = 256;
struct StencilGrid {
  int blocks, threads, sh;
};
// tpb_req: requested site tiles per workgroup (0: enough for >= 4 waves);
// xcd: apply the XCD-aware block order
inline StencilGrid stencil_grid(int nsite, int ngrp, int tpb_req, int xcd) {
  const int maxw = kStencilMaxThreads / 64;
  // column groups per workgroup: the largest divisor of ngrp that fits, so no
  // wave of a workgroup is left without columns
  int gw = 1;
  for (int d = maxw; d > 1; --d)
    if (ngrp % d == 0) {
      gw = d;
      break;
    }
  int tpb = tpb_req > 0 ? tpb_req : (gw >= 4 ? 1 : 4 / gw);
  if (tpb * gw > maxw) tpb = maxw / gw;
  if (tpb < 1) tpb = 1;
  const int nchunk = (ngrp + gw - 1) / gw;
  const int ntile = (nsite + 63) / 64;
  return {((ntile + tpb - 1) / tpb) * nchunk, 64 * gw * tpb, gw | (tpb << 8) | ((xcd ? 1 : 0) << 16)};
}

}  // namespace lq
