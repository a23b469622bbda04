// Two-level aggregation multigrid for the Wilson-type operators (sec. 2.1,
// Table 2's multigrid inverter): transfer operators between the fine lattice
// and the coarse lattice of aggregates, the coarse (Galerkin) stencil, and the
// setup kernels that build them.
//
// Coarse vectors hold n2 = 2 nv complex numbers per coarse site, index
// d = s nv + j (s = 0: chirality +, spins 0 and 1; s = 1: chirality -).  They
// are stored as a Wilson-shaped field with K = n2 / 12 pseudo-sites per coarse
// site (npar = 1, Vh = K Vc), so the vector kernels of the solvers run on them
// unchanged; component d of coarse site Y is component d % 12 of pseudo-site
// Y K + d / 12.
//
// The basis Q[Vc][B][2][nv][6] holds, per aggregate, in-block site, chirality
// and vector, the six spin-colour components of that chirality (orthonormal
// over each (aggregate, chirality) after launch_mg_orth).  The coarse operator
// Dc[Vc][9][n2 (column k)][n2 (row i)]: direction 0 is the aggregate itself,
// 1 + 2 mu couples to Y + mu and 2 + 2 mu to Y - mu; rows are contiguous so
// that the threads of a coarse site read a column in one pass.
#include <cstdlib>

#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

namespace {

typedef float mg_f4 __attribute__((ext_vector_type(4)));
typedef double mg_d4 __attribute__((ext_vector_type(4)));

// the coarse stencil and the prolongation on the matrix cores unless LQ_MG_VALU is set
inline bool mg_use_mfma() {
  static const bool v = getenv("LQ_MG_VALU") == nullptr;
  return v;
}

template <int P> struct CxT;
template <> struct CxT<64> { using T = double2; using R = double; };
template <> struct CxT<32> { using T = float2; using R = float; };

// one complex number of a coarse vector, at pseudo-site q of block blk
template <int P> struct CIO;
template <> struct CIO<64> {
  static __device__ __forceinline__ cx<double> ld(const FieldRef& f, int64_t blk, int q, int c) {
    const double2 v = ((const double2*)f.data)[tix(blk, c, 12, q, f.Vh)];
    return {v.x, v.y};
  }
  static __device__ __forceinline__ void st(const FieldRef& f, int64_t blk, int q, int c, cx<double> v) {
    ((double2*)f.data)[tix(blk, c, 12, q, f.Vh)] = make_double2(v.re, v.im);
  }
};
template <> struct CIO<32> {
  static __device__ __forceinline__ cx<float> ld(const FieldRef& f, int64_t blk, int q, int c) {
    const float2 v = ((const float2*)f.data)[2 * tix(blk, c >> 1, 6, q, f.Vh) + (c & 1)];
    return {v.x, v.y};
  }
  static __device__ __forceinline__ void st(const FieldRef& f, int64_t blk, int q, int c, cx<float> v) {
    ((float2*)f.data)[2 * tix(blk, c >> 1, 6, q, f.Vh) + (c & 1)] = make_float2(v.re, v.im);
  }
};
// component d of aggregate Y in column col: the aggregate's parity block
// (npar = 2, or the one stored parity of an npar = 1 vector) and its
// checkerboard index, K pseudo-sites per aggregate
template <int P>
__device__ __forceinline__ cx<typename CxT<P>::R> cld(const FieldRef& f, const MgGeom& m, int col, int Y, int d) {
  const int v = m.cmap[Y];
  const int64_t blk = (int64_t)col * f.npar + (f.npar == 2 ? (v >> 30) & 1 : 0);
  return CIO<P>::ld(f, blk, (v & 0x3fffffff) * m.K + d / 12, d % 12);
}
template <int P>
__device__ __forceinline__ void cst(const FieldRef& f, const MgGeom& m, int col, int Y, int d,
                                    cx<typename CxT<P>::R> x) {
  const int v = m.cmap[Y];
  const int64_t blk = (int64_t)col * f.npar + (f.npar == 2 ? (v >> 30) & 1 : 0);
  CIO<P>::st(f, blk, (v & 0x3fffffff) * m.K + d / 12, d % 12, x);
}

// the six components of chirality s of a fine Wilson site (FP64 / FP32 layouts)
template <int P> struct HalfIO;
template <> struct HalfIO<64> {
  static __device__ __forceinline__ void ld(const FieldRef& f, int64_t blk, int cb, int s, cx<double>* v) {
    const double2* p = (const double2*)f.data;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double2 d = p[tix(blk, 6 * s + c, 12, cb, f.Vh)];
      v[c] = {d.x, d.y};
    }
  }
  static __device__ __forceinline__ void st(const FieldRef& f, int64_t blk, int cb, int s, const cx<double>* v) {
    double2* p = (double2*)f.data;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[tix(blk, 6 * s + c, 12, cb, f.Vh)] = make_double2(v[c].re, v[c].im);
  }
};
template <> struct HalfIO<32> {
  static __device__ __forceinline__ void ld(const FieldRef& f, int64_t blk, int cb, int s, cx<float>* v) {
    const float4* p = (const float4*)f.data;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 d = p[tix(blk, 3 * s + k, 6, cb, f.Vh)];
      v[2 * k] = {d.x, d.y};
      v[2 * k + 1] = {d.z, d.w};
    }
  }
  static __device__ __forceinline__ void st(const FieldRef& f, int64_t blk, int cb, int s, const cx<float>* v) {
    float4* p = (float4*)f.data;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      p[tix(blk, 3 * s + k, 6, cb, f.Vh)] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
  }
};


__device__ __forceinline__ void fine_site(const MgGeom& m, int yb, int& cb, int& par) {
  const int v = m.fine[yb];
  cb = v & 0x3fffffff;
  par = (v >> 30) & 1;
}

// ---------------------------------------------------------------- transfers
// restriction: coarse(col, Y, s nv + j) = sum over the aggregate's sites of
// q_{Y,s,j}^dag v_s; one thread per (Y, s, j), CB columns per thread (the
// basis is read once per CB columns)
template <int PF, int PC, int CB>
__global__ void __launch_bounds__(256) mg_restrict_kernel(MgGeom m, const void* Qv, FieldRef fine, FieldRef coarse,
                                                           int ncol) {
  using R = typename CxT<PF>::R;
  // four waves split the aggregate's sites, their sums meet in LDS
  __shared__ cx<R> part[3][64][CB];
  const int Y = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n2 = 2 * m.nv;
  const int t = lane < n2 ? lane : n2 - 1;  // idle lanes repeat the last row and store nothing
  const int s = t / m.nv, j = t - s * m.nv;
  const int col0 = blockIdx.y * CB;
  const int nc = min(CB, ncol - col0);
  const cx<R>* Q = (const cx<R>*)Qv;
  cx<R> acc[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) acc[c] = {0, 0};
  const int bq = (m.B + 3) >> 2, b0 = wv * bq, b1 = min(m.B, b0 + bq);
  for (int b = b0; b < b1; ++b) {
    const int yb = Y * m.B + b;
    int cb, par;
    fine_site(m, yb, cb, par);
    const cx<R>* q = Q + (((int64_t)yb * 2 + s) * m.nv + j) * 6;
    cx<R> qv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) qv[c] = q[c];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) {
      if (cc < nc) {
        cx<R> v[6];
        HalfIO<PF>::ld(fine, (int64_t)(col0 + cc) * 2 + par, cb, s, v);
#pragma unroll
        for (int c = 0; c < 6; ++c) fmac(acc[cc], qv[c], v[c]);
      }
    }
  }
  if (wv > 0)
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) part[wv - 1][lane][cc] = acc[cc];
  __syncthreads();
  if (wv > 0 || lane >= n2) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) acc[cc] = acc[cc] + part[w][lane][cc];
  using RC = typename CxT<PC>::R;
#pragma unroll
  for (int cc = 0; cc < CB; ++cc)
    if (cc < nc) cst<PC>(coarse, m, col0 + cc, Y, t, cx<RC>{(RC)acc[cc].re, (RC)acc[cc].im});
}

// prolongation: fine(col, y)_s = sum_j coarse(col, Y(y), s nv + j) q_{Y,s,j}(y);
// one thread per (aggregate site, chirality), CB columns per thread
template <int PC, int PF, int CB>
__global__ void __launch_bounds__(256) mg_prolong_kernel(MgGeom m, FieldRef coarse, const void* Qv, FieldRef fine,
                                                          int ncol) {
  using R = typename CxT<PF>::R;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m.Vc * m.B * 2) return;
  const int yb = (int)(gid >> 1), s = (int)(gid & 1);
  const int Y = yb / m.B;
  const int col0 = blockIdx.y * CB;
  const int nc = min(CB, ncol - col0);
  const cx<R>* q = (const cx<R>*)Qv + (int64_t)yb * 2 * m.nv * 6 + (int64_t)s * m.nv * 6;
  cx<R> acc[CB][6];
#pragma unroll
  for (int cc = 0; cc < CB; ++cc)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[cc][c] = {0, 0};
  for (int j = 0; j < m.nv; ++j) {
    cx<R> qv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) qv[c] = q[j * 6 + c];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) {
      if (cc < nc) {
        const auto a = cld<PC>(coarse, m, col0 + cc, Y, s * m.nv + j);
        const cx<R> ar = {(R)a.re, (R)a.im};
#pragma unroll
        for (int c = 0; c < 6; ++c) fma(acc[cc][c], qv[c], ar);
      }
    }
  }
  int cb, par;
  fine_site(m, yb, cb, par);
#pragma unroll
  for (int cc = 0; cc < CB; ++cc)
    if (cc < nc) HalfIO<PF>::st(fine, (int64_t)(col0 + cc) * 2 + par, cb, s, acc[cc]);
}

// Prolongation into FP32 fine vectors on the matrix cores: for one
// (aggregate, chirality) the fine block F (6 B rows (site, component) x 12
// columns) is Q (6 B x nv) times the coarse block V (nv x 12), as the real
// product [Qr | Qi] [[Vr, Vi], [-Vi, Vr]] = [Fr | Fi] with
// v_mfma_f32_16x16x4f32: 16-row tiles of F, two 16-column tiles for the 24
// real columns, k (the vector index) in groups of 4 padded to nv rounded up.
// One workgroup of four waves per (aggregate, chirality), V staged in LDS; each
// wave takes every fourth row tile and stages its output tile in LDS to write
// complex pairs.  Lane layouts as in the coarse stencil.
template <int PC>
__global__ void __launch_bounds__(256) mg_prolong_mfma_kernel(MgGeom m, FieldRef coarse, const float2* Q,
                                                               FieldRef fine, int ncol) {
  __shared__ float2 sv[32 * 12];
  __shared__ float so[4][16][25];
  const int Y = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r16 = lane & 15, q = lane >> 4;
  const int col0 = blockIdx.y * 12;
  const int nc = min(12, ncol - col0);
  const int nv = m.nv, nkg = (nv + 3) >> 2;
  for (int e = tid; e < 32 * 12; e += blockDim.x) {
    const int j = e / 12, cc = e - j * 12;
    float2 v = make_float2(0.f, 0.f);
    if (j < nv && cc < nc) {
      const auto a = cld<PC>(coarse, m, col0 + cc, Y, s * nv + j);
      v = make_float2((float)a.re, (float)a.im);
    }
    sv[e] = v;
  }
  __syncthreads();
  // B operands of this lane for each k-group (the same for every row tile)
  float bR[8][2], bI[8][2];
#pragma unroll
  for (int kg = 0; kg < 8; ++kg) {
    const int k = 4 * kg + q;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int n = 16 * t + r16;
      const float2 xv = n < 24 ? sv[k * 12 + (n < 12 ? n : n - 12)] : make_float2(0.f, 0.f);
      bR[kg][t] = n < 12 ? xv.x : (n < 24 ? xv.y : 0.f);
      bI[kg][t] = n < 12 ? -xv.y : (n < 24 ? xv.x : 0.f);
    }
  }
  const int rows = 6 * m.B, ntile = (rows + 15) >> 4;
  const int64_t sstride = (int64_t)2 * nv * 6;  // complex entries between in-block sites
  const float2* QY = Q + (int64_t)Y * m.B * sstride + (int64_t)s * nv * 6;
  for (int tile = wv; tile < ntile; tile += 4) {
    const int row = 16 * tile + r16;
    const int b = row / 6, c = row - 6 * b;
    mg_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kg = 0; kg < 8; ++kg) {
      if (kg < nkg) {
        const int j = 4 * kg + q;
        const float2 av = (row < rows && j < nv) ? QY[(int64_t)b * sstride + j * 6 + c] : make_float2(0.f, 0.f);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bR[kg][0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bR[kg][1], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bI[kg][0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bI[kg][1], acc1, 0, 0, 0);
      }
    }
    // the wave's output tile through LDS: so[wave][row in tile][real column]
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int n = 16 * u + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (n < 24) so[wv][4 * q + i][n] = u == 0 ? acc0[i] : acc1[i];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < 16 * 12; e += 64) {
      const int rr = e / 12, cc = e - rr * 12;
      const int orow = 16 * tile + rr;
      if (cc < nc && orow < rows) {
        const int ob = orow / 6, oc = orow - 6 * ob;
        int cb, par;
        fine_site(m, Y * m.B + ob, cb, par);
        const int comp = 6 * s + oc;
        float2* p = (float2*)fine.data;
        p[2 * tix((int64_t)(col0 + cc) * 2 + par, comp >> 1, 6, cb, fine.Vh) + (comp & 1)] =
            make_float2(so[wv][rr][cc], so[wv][rr][12 + cc]);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------- coarse stencil
// The generic coarse stencil over the aggregates Y of parity par_out (2: all):
//   out(Y) = a x(Y) + sgn sum_{d = d0}^{d0 + nd - 1} M[Y][d] in(N_d(Y))
// with M[Y][d] an (n2 x n2) block stored by columns (direction 0: the
// aggregate itself).  One wave per aggregate, thread i = row; the input block
// of each direction (n2 x NCB columns) is staged in LDS, so the wave streams
// its blocks from HBM once per NCB columns.  (Prefetching the next direction's
// block into registers measured slower: loads complete in order, so the first
// matrix load of a direction waits for them.)
template <int P, int NCB>
__global__ void __launch_bounds__(64) mg_stencil_kernel(MgGeom m, const void* Mv, int d0, int nd, FieldRef in,
                                                         FieldRef out, FieldRef x, double a, double sgn,
                                                         int par_out, int ncol) {
  using R = typename CxT<P>::R;
  __shared__ cx<R> sin_[64 * NCB];
  const int Y = par_out == 2 ? blockIdx.x : m.csite[par_out * (m.Vc / 2) + blockIdx.x];
  const int i = threadIdx.x, n2 = 2 * m.nv;
  const int col0 = blockIdx.y * NCB;
  const int nc = min(NCB, ncol - col0);
  cx<R> acc[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) acc[c] = {0, 0};
  for (int d = d0; d < d0 + nd; ++d) {
    const int Yn = d == 0 ? Y : m.nbr[Y * 8 + d - 1];
    __syncthreads();  // the previous direction's block is no longer read
    for (int e = i; e < n2 * NCB; e += 64) {
      const int k = e / NCB, cc = e - k * NCB;
      sin_[e] = cc < nc ? cld<P>(in, m, col0 + cc, Yn, k) : cx<R>{0, 0};
    }
    __syncthreads();
    if (i < n2) {
      const cx<R>* M = (const cx<R>*)Mv + ((int64_t)Y * 9 + d) * n2 * n2 + i;
#pragma unroll 8
      for (int k = 0; k < n2; ++k) {
        const cx<R> w = M[(int64_t)k * n2];
#pragma unroll
        for (int cc = 0; cc < NCB; ++cc) fma(acc[cc], w, sin_[k * NCB + cc]);
      }
    }
  }
  if (i < n2) {
#pragma unroll
    for (int cc = 0; cc < NCB; ++cc) {
      if (cc < nc) {
        cx<R> o = {(R)sgn * acc[cc].re, (R)sgn * acc[cc].im};
        if (a != 0.0) o = o + (R)a * cld<P>(x, m, col0 + cc, Y, i);
        cst<P>(out, m, col0 + cc, Y, i, o);
      }
    }
  }
}

// The same stencil on the matrix cores, 12 columns per workgroup: per
// direction the complex product Y = M X (n2 x n2 times n2 x 12) is the real
// product [Mr | Mi] [[Xr, Xi], [-Xi, Xr]] = [Yr | Yi], done as 16x16x4 MFMA
// steps (v_mfma_f32_16x16x4f32, or v_mfma_f64_16x16x4f64 for the FP64
// stencil).  One wave per 16-row tile of M (n2 / 16 waves, the last tile
// padded), the 24 real output columns in two 16-column tiles (8 padding
// columns), k in groups of 4; the real and imaginary parts of one loaded
// matrix element feed the Mr and the Mi step of the same k.  A wave issues all
// its matrix loads of a direction before its first MFMA.  Lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; of the output tile it holds
// D[4 (l / 16) + i][l % 16], i = 0..3, in FP32, and D[4 i + l / 16][l % 16]
// in FP64.
template <int P> struct MfmaT;
template <> struct MfmaT<32> {
  using R = float;
  using C2 = float2;
  using V4 = mg_f4;
  static __device__ __forceinline__ V4 mma(R a, R b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int drow(int q, int i) { return 4 * q + i; }
};
template <> struct MfmaT<64> {
  using R = double;
  using C2 = double2;
  using V4 = mg_d4;
  static __device__ __forceinline__ V4 mma(R a, R b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int drow(int q, int i) { return 4 * i + q; }
};

template <int P>
__global__ void __launch_bounds__(256) mg_stencil_mfma_kernel(MgGeom m, const void* Mv, int d0, int nd, FieldRef in,
                                                               FieldRef out, FieldRef x, double a, double sgn,
                                                               int par_out, int ncol) {
  using T = MfmaT<P>;
  using R = typename T::R;
  using C2 = typename T::C2;
  __shared__ C2 sx[64 * 12];
  __shared__ R so[2][64][13];
  const int Y = par_out == 2 ? blockIdx.x : m.csite[par_out * (m.Vc / 2) + blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r16 = lane & 15, q = lane >> 4;
  const int n2 = 2 * m.nv, nkg = n2 >> 2;  // n2 <= 60: at most 15 k-groups
  const int col0 = blockIdx.y * 12;
  const int nc = min(12, ncol - col0);
  const int row = 16 * wv + r16;
  typename T::V4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  for (int d = d0; d < d0 + nd; ++d) {
    const int Yn = d == 0 ? Y : m.nbr[Y * 8 + d - 1];
    // this wave's matrix elements of the direction: A[row][4 kg + q], kg < nkg
    const C2* M = (const C2*)Mv + ((int64_t)Y * 9 + d) * n2 * n2 + row;
    C2 av[15];
#pragma unroll
    for (int kg = 0; kg < 15; ++kg) {
      if (kg < nkg && row < n2) av[kg] = M[(int64_t)(4 * kg + q) * n2];
      else av[kg].x = av[kg].y = 0;
    }
    __syncthreads();
    for (int e = tid; e < n2 * 12; e += blockDim.x) {
      const int k = e / 12, cc = e - k * 12;
      const cx<R> v = cc < nc ? cld<P>(in, m, col0 + cc, Yn, k) : cx<R>{0, 0};
      sx[e].x = v.re;
      sx[e].y = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int kg = 0; kg < 15; ++kg) {
      if (kg < nkg) {
        const int k = 4 * kg + q;
        R bR[2], bI[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int n = 16 * t + r16;
          C2 xv;
          xv.x = xv.y = 0;
          if (n < 24) xv = sx[k * 12 + (n < 12 ? n : n - 12)];
          bR[t] = n < 12 ? xv.x : (n < 24 ? xv.y : (R)0);
          bI[t] = n < 12 ? -xv.y : (n < 24 ? xv.x : (R)0);
        }
        acc0 = T::mma(av[kg].x, bR[0], acc0);
        acc1 = T::mma(av[kg].x, bR[1], acc1);
        acc0 = T::mma(av[kg].y, bI[0], acc0);
        acc1 = T::mma(av[kg].y, bI[1], acc1);
      }
    }
  }
  // D tiles -> [re / im][row][column] in LDS, then one complex output per (row, column)
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int n = 16 * u + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * wv + T::drow(q, i);
      const R v = u == 0 ? acc0[i] : acc1[i];
      if (n < 24 && r < 64) so[n < 12 ? 0 : 1][r][n < 12 ? n : n - 12] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < n2 * nc; e += blockDim.x) {
    const int r = e / nc, cc = e - r * nc;
    cx<R> o = {(R)sgn * so[0][r][cc], (R)sgn * so[1][r][cc]};
    if (a != 0.0) o = o + (R)a * cld<P>(x, m, col0 + cc, Y, r);
    cst<P>(out, m, col0 + cc, Y, r, o);
  }
}

// ---------------------------------------------------------------- block Gram-Schmidt
// Classical Gram-Schmidt step of the outer flexible GCR on k <= 8 earlier
// directions: c_j = <W_j, w> for all j in one pass over w (per-block partials,
// summed in block order: deterministic), then w -= sum_j c_j W_j and
// z -= sum_j c_j Z_j in one pass.
struct MgVecSet {
  FieldRef f[8];
};

template <int P>
__global__ void __launch_bounds__(256) mg_mdot_kernel(MgVecSet W, int k, FieldRef w, int npar, double* partial) {
  using R = typename CxT<P>::R;
  __shared__ double sm[4][16];
  const int col = blockIdx.y, ncol = gridDim.y;
  const int64_t n = (int64_t)npar * w.Vh;
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int par = (int)(i / w.Vh), cb = (int)(i - (int64_t)par * w.Vh);
    const int64_t blk = (int64_t)col * npar + par;
    cx<R> b[12];
    IO<P, 12>::load(w, blk, cb, b);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < k) {
        cx<R> a[12];
        IO<P, 12>::load(W.f[j], blk, cb, a);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          acc[2 * j] += (double)a[c].re * (double)b[c].re + (double)a[c].im * (double)b[c].im;
          acc[2 * j + 1] += (double)a[c].re * (double)b[c].im - (double)a[c].im * (double)b[c].re;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j)
    for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < 16; ++j) sm[wv][j] = acc[j];
  __syncthreads();
  if ((int)threadIdx.x < 2 * k) {
    const int j = threadIdx.x;
    double v = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v += sm[q][j];
    partial[((int64_t)(j >> 1) * ncol + col) * gridDim.x * 2 + (int64_t)blockIdx.x * 2 + (j & 1)] = v;
  }
}

__global__ void mg_mdot_sum_kernel(const double* partial, int k, int ncol, int gridx, double* coef) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * ncol) return;
  const double* p = partial + (int64_t)t * gridx * 2;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < gridx; ++b) {
    re += p[2 * b];
    im += p[2 * b + 1];
  }
  coef[2 * t] = re;
  coef[2 * t + 1] = im;
}

template <int P>
__global__ void __launch_bounds__(256) mg_maxmy_kernel(MgVecSet W, MgVecSet Z, int k, FieldRef w, FieldRef z,
                                                        int npar, const double* coef) {
  using R = typename CxT<P>::R;
  const int col = blockIdx.y, ncol = gridDim.y;
  const int64_t n = (int64_t)npar * w.Vh;
  cx<R> c[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    c[j] = j < k ? cx<R>{(R)coef[2 * (j * ncol + col)], (R)coef[2 * (j * ncol + col) + 1]} : cx<R>{0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int par = (int)(i / w.Vh), cb = (int)(i - (int64_t)par * w.Vh);
    const int64_t blk = (int64_t)col * npar + par;
    cx<R> x[12], y[12], a[12];
    IO<P, 12>::load(w, blk, cb, x);
    IO<P, 12>::load(z, blk, cb, y);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < k) {
        IO<P, 12>::load(W.f[j], blk, cb, a);
#pragma unroll
        for (int q = 0; q < 12; ++q) x[q] = x[q] - c[j] * a[q];
        IO<P, 12>::load(Z.f[j], blk, cb, a);
#pragma unroll
        for (int q = 0; q < 12; ++q) y[q] = y[q] - c[j] * a[q];
      }
    }
    IO<P, 12>::store(w, blk, cb, x);
    IO<P, 12>::store(z, blk, cb, y);
  }
}

// ---------------------------------------------------------------- setup
// Q[:, :, s, j, :] = chirality-s half of fine column j (FP64)
__global__ void __launch_bounds__(256) mg_gather_kernel(MgGeom m, FieldRef fine, double2* Q) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)m.Vc * m.B * 2 * m.nv;
  if (gid >= n) return;
  const int j = (int)(gid % m.nv);
  const int s = (int)((gid / m.nv) & 1);
  const int yb = (int)(gid / (2 * m.nv));
  int cb, par;
  fine_site(m, yb, cb, par);
  cx<double> v[6];
  HalfIO<64>::ld(fine, (int64_t)j * 2 + par, cb, s, v);
  double2* q = Q + (((int64_t)yb * 2 + s) * m.nv + j) * 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) q[c] = make_double2(v[c].re, v[c].im);
}

__device__ __forceinline__ double2 block_sum2(double2 v, double2* sm) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();  // sm is free again
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) {
    r.x += sm[k].x;
    r.y += sm[k].y;
  }
  return r;
}

// Gram-Schmidt in vector order, two passes, on every (aggregate, chirality):
// one workgroup of 256 threads each; vectors of B*6 complex numbers
__global__ void __launch_bounds__(256) mg_orth_kernel(MgGeom m, double2* Q, int* bad) {
  __shared__ double2 sm[4];
  const int Y = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int n = m.B * 6;
  const int64_t sstride = (int64_t)2 * m.nv * 6;  // between in-block sites
  auto at = [&](int j, int e) -> double2& {
    const int b = e / 6, c = e - 6 * (e / 6);
    return Q[((int64_t)(Y * m.B + b)) * sstride + ((int64_t)s * m.nv + j) * 6 + c];
  };
  for (int j = 0; j < m.nv; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        double2 d = make_double2(0.0, 0.0);
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
          const double2 a = at(i, e), b = at(j, e);
          d.x += a.x * b.x + a.y * b.y;
          d.y += a.x * b.y - a.y * b.x;
        }
        d = block_sum2(d, sm);
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
          const double2 a = at(i, e);
          double2& b = at(j, e);
          b.x -= d.x * a.x - d.y * a.y;
          b.y -= d.x * a.y + d.y * a.x;
        }
        __syncthreads();
      }
    }
    double2 nn = make_double2(0.0, 0.0);
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const double2 a = at(j, e);
      nn.x += a.x * a.x + a.y * a.y;
    }
    nn = block_sum2(nn, sm);
    const double inv = nn.x > 0.0 ? 1.0 / sqrt(nn.x) : 0.0;
    if (nn.x <= 0.0 && threadIdx.x == 0) atomicAdd(bad, 1);
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      double2& a = at(j, e);
      a.x *= inv;
      a.y *= inv;
    }
    __syncthreads();
  }
}

// Columns k0.. of Dc from D applied to the probe sources of class cls: an
// aggregate of class cls restricts its whole block into the self term; an
// aggregate whose class differs in the bit of direction mu only receives the
// hops of its two mu-neighbours, the one at Y - mu on its lower mu-face and
// the one at Y + mu on its upper mu-face (blocks are at least 2 sites deep, so
// the faces are disjoint).  Other aggregates receive nothing.
__global__ void __launch_bounds__(256) mg_probe_restrict_kernel(MgGeom m, const double2* Q, FieldRef fine, int ncol,
                                                                 int k0, int cls, double2* Dc) {
  // four waves split the aggregate's sites; the ncol (<= 12) probe columns are
  // taken together so that the basis is read once; partial sums meet in LDS
  __shared__ double2 part[3][64][2][12];
  const int Y = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n2 = 2 * m.nv;
  const int bits = m.cpar[Y] ^ cls;
  if (bits & (bits - 1)) return;  // the whole workgroup: no aggregate of this class is next to Y
  const int mu = bits ? __ffs(bits) - 1 : -1;
  const int t = lane < n2 ? lane : n2 - 1;
  const int s = t / m.nv, j = t - s * m.nv;
  cx<double> lo[12], hi[12];
#pragma unroll
  for (int kk = 0; kk < 12; ++kk) lo[kk] = hi[kk] = cx<double>{0, 0};
  const int bq = (m.B + 3) >> 2, b0 = wv * bq, b1 = min(m.B, b0 + bq);
  for (int b = b0; b < b1; ++b) {
    const int yb = Y * m.B + b;
    const int fb = m.face[yb];
    const bool in_lo = mu < 0 || (fb >> (2 * mu)) & 1;
    const bool in_hi = mu >= 0 && (fb >> (2 * mu + 1)) & 1;
    if (!in_lo && !in_hi) continue;
    int cb, par;
    fine_site(m, yb, cb, par);
    const double2* q = Q + (((int64_t)yb * 2 + s) * m.nv + j) * 6;
    cx<double> qv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) qv[c] = cx<double>{q[c].x, q[c].y};
#pragma unroll
    for (int kk = 0; kk < 12; ++kk) {
      if (kk < ncol) {
        cx<double> v[6];
        HalfIO<64>::ld(fine, (int64_t)kk * 2 + par, cb, s, v);
        cx<double> acc = {0, 0};
#pragma unroll
        for (int c = 0; c < 6; ++c) fmac(acc, qv[c], v[c]);
        if (in_lo) lo[kk] = lo[kk] + acc;
        if (in_hi) hi[kk] = hi[kk] + acc;
      }
    }
  }
  if (wv > 0)
#pragma unroll
    for (int kk = 0; kk < 12; ++kk) {
      part[wv - 1][lane][0][kk] = make_double2(lo[kk].re, lo[kk].im);
      part[wv - 1][lane][1][kk] = make_double2(hi[kk].re, hi[kk].im);
    }
  __syncthreads();
  if (wv > 0 || lane >= n2) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int kk = 0; kk < 12; ++kk) {
      lo[kk] = lo[kk] + cx<double>{part[w][lane][0][kk].x, part[w][lane][0][kk].y};
      hi[kk] = hi[kk] + cx<double>{part[w][lane][1][kk].x, part[w][lane][1][kk].y};
    }
  for (int kk = 0; kk < ncol; ++kk) {
    const int k = k0 + kk;
    if (mu < 0) {
      Dc[(((int64_t)Y * 9) * n2 + k) * n2 + t] = make_double2(lo[kk].re, lo[kk].im);
    } else {
      Dc[(((int64_t)Y * 9 + 2 + 2 * mu) * n2 + k) * n2 + t] = make_double2(lo[kk].re, lo[kk].im);
      Dc[(((int64_t)Y * 9 + 1 + 2 * mu) * n2 + k) * n2 + t] = make_double2(hi[kk].re, hi[kk].im);
    }
  }
}

// the probe fine vectors directly: column kk is chirality s = (k0 + kk) / nv of
// basis vector j = (k0 + kk) % nv on the aggregates of class cls, zero elsewhere
__global__ void __launch_bounds__(256) mg_probe_fine_kernel(MgGeom m, const double2* Q, FieldRef fine, int ncol,
                                                             int k0, int cls) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m.Vc * m.B * ncol) return;
  const int yb = (int)(gid % ((int64_t)m.Vc * m.B)), kk = (int)(gid / ((int64_t)m.Vc * m.B));
  const int Y = yb / m.B;
  const int d = k0 + kk, s = d / m.nv, j = d - s * m.nv;
  cx<double> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = cx<double>{0, 0};
  if (m.cpar[Y] == cls) {
    const double2* q = Q + (((int64_t)yb * 2 + s) * m.nv + j) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) v[6 * s + c] = cx<double>{q[c].x, q[c].y};
  }
  int cb, par;
  fine_site(m, yb, cb, par);
  IO<64, 12>::store(fine, (int64_t)kk * 2 + par, cb, v);
}

__global__ void __launch_bounds__(256) mg_narrow_kernel(const double2* src, float2* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = src[i];
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

// splitmix64 (Steele, Lea, Flood 2014) of (seed, element): uniform in [-1, 1)
__device__ __forceinline__ double mix_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void __launch_bounds__(256) mg_random_kernel(FieldRef fine, int ncol, uint64_t seed) {
  const int64_t n = (int64_t)ncol * 2 * fine.Vh;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = i / fine.Vh;
    const int cb = (int)(i - blk * fine.Vh);
    cx<double> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const uint64_t e = ((uint64_t)i * 12 + c) * 2;
      v[c] = {mix_uniform(seed, e), mix_uniform(seed, e + 1)};
    }
    IO<64, 12>::store(fine, blk, cb, v);
  }
}

// A^{-1} of every aggregate's self block A = Dc[Y][0] (FP64 Gauss-Jordan with
// partial pivoting on [A | 1], one wave per aggregate, in a global workspace of
// n2 x 2 n2 complex per aggregate) into Ahat[Y][0]
__global__ void __launch_bounds__(64) mg_site_inverse_kernel(MgGeom m, const double2* Dc, double2* Ahat,
                                                              double2* work, int* bad) {
  const int Y = blockIdx.x, t = threadIdx.x, n2 = 2 * m.nv, w = 2 * n2;
  double2* G = work + (int64_t)Y * n2 * w;  // [row][2 n2]
  __shared__ int piv;
  const double2* A = Dc + (int64_t)Y * 9 * n2 * n2;  // column k at A + k n2
  for (int e = t; e < n2 * w; e += 64) {
    const int r = e / w, c = e - r * w;
    G[e] = c < n2 ? A[(int64_t)c * n2 + r] : make_double2(c - n2 == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < n2; ++k) {
    if (t == 0) {
      int p = k;
      double best = -1.0;
      for (int r = k; r < n2; ++r) {
        const double2 v = G[r * w + k];
        const double a2 = v.x * v.x + v.y * v.y;
        if (a2 > best) {
          best = a2;
          p = r;
        }
      }
      piv = p;
      if (!(best > 0.0)) atomicAdd(bad, 1);
    }
    __syncthreads();
    const int p = piv;
    if (p != k)
      for (int c = t; c < w; c += 64) {
        const double2 u = G[k * w + c];
        G[k * w + c] = G[p * w + c];
        G[p * w + c] = u;
      }
    __syncthreads();
    const double2 d = G[k * w + k];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 inv = make_double2(d.x / dd, -d.y / dd);
    __syncthreads();
    for (int c = t; c < w; c += 64) {
      const double2 u = G[k * w + c];
      G[k * w + c] = make_double2(u.x * inv.x - u.y * inv.y, u.x * inv.y + u.y * inv.x);
    }
    __syncthreads();
    for (int e = t; e < n2 * w; e += 64) {
      const int r = e / w, c = e - r * w;
      if (r == k) continue;
      const double2 f = G[r * w + k];
      const double2 u = G[k * w + c];
      if (c == k) continue;  // column k of row r is cleared below, after every row has read it
      G[r * w + c] = make_double2(G[r * w + c].x - (f.x * u.x - f.y * u.y), G[r * w + c].y - (f.x * u.y + f.y * u.x));
    }
    __syncthreads();
    for (int r = t; r < n2; r += 64)
      if (r != k) G[r * w + k] = make_double2(0.0, 0.0);
    __syncthreads();
  }
  double2* out = Ahat + (int64_t)Y * 9 * n2 * n2;
  for (int e = t; e < n2 * n2; e += 64) {
    const int r = e / n2, c = e - r * n2;
    out[(int64_t)c * n2 + r] = G[r * w + n2 + c];
  }
}

// Ahat[Y][d] = A^{-1}(Y) Dc[Y][d] for the eight hops (blocks stored by columns):
// thread i computes row i of every column
__global__ void __launch_bounds__(64) mg_site_mul_kernel(MgGeom m, const double2* Dc, double2* Ahat) {
  const int Y = blockIdx.x, d = 1 + blockIdx.y, i = threadIdx.x, n2 = 2 * m.nv;
  if (i >= n2) return;
  const double2* Ai = Ahat + (int64_t)Y * 9 * n2 * n2;          // A^{-1}, column j at Ai + j n2
  const double2* M = Dc + ((int64_t)Y * 9 + d) * n2 * n2;        // column k at M + k n2
  double2* C = Ahat + ((int64_t)Y * 9 + d) * n2 * n2;
  for (int k = 0; k < n2; ++k) {
    cx<double> acc = {0, 0};
    for (int j = 0; j < n2; ++j) {
      const double2 a = Ai[(int64_t)j * n2 + i], b = M[(int64_t)k * n2 + j];
      fma(acc, cx<double>{a.x, a.y}, cx<double>{b.x, b.y});
    }
    C[(int64_t)k * n2 + i] = make_double2(acc.re, acc.im);
  }
}

inline int grid_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 1 << 20); }

}  // namespace

int launch_mg_restrict(const MgGeom& m, int pf, const void* Q, FieldRef fine, int pc, FieldRef coarse, int ncol,
                       hipStream_t s) {
  if (ncol <= 0) return 0;
  if (2 * m.nv > 64) return -1;
  const bool wide = ncol > 4;
  dim3 grid(m.Vc, wide ? (ncol + 11) / 12 : (ncol + 3) / 4), block(256);
#define LQ_MG_R(PF, PC)                                                                              \
  if (pf == PF && pc == PC) {                                                                        \
    if (wide) mg_restrict_kernel<PF, PC, 12><<<grid, block, 0, s>>>(m, Q, fine, coarse, ncol);       \
    else mg_restrict_kernel<PF, PC, 4><<<grid, block, 0, s>>>(m, Q, fine, coarse, ncol);             \
    return hipGetLastError() == hipSuccess ? 0 : -2;                                                 \
  }
  LQ_MG_R(64, 64)
  LQ_MG_R(32, 64)
  LQ_MG_R(32, 32)
  LQ_MG_R(64, 32)
#undef LQ_MG_R
  return -1;
}

int launch_mg_prolong(const MgGeom& m, int pc, FieldRef coarse, int pf, const void* Q, FieldRef fine, int ncol,
                      hipStream_t s) {
  if (ncol <= 0) return 0;
  const int64_t n = (int64_t)m.Vc * m.B * 2;
  // twelve columns per thread for FP32 fine vectors (the V-cycle); four for FP64 (setup probes), whose
  // twelve-column version needs all 256 registers
  const bool wide = ncol > 4 && pf == 32;
  if (wide && mg_use_mfma() && m.nv <= 32) {
    dim3 g2(m.Vc * 2, (ncol + 11) / 12);
    if (pc == 64) mg_prolong_mfma_kernel<64><<<g2, 256, 0, s>>>(m, coarse, (const float2*)Q, fine, ncol);
    else mg_prolong_mfma_kernel<32><<<g2, 256, 0, s>>>(m, coarse, (const float2*)Q, fine, ncol);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
  dim3 grid((unsigned)((n + 255) / 256), wide ? (ncol + 11) / 12 : (ncol + 3) / 4), block(256);
#define LQ_MG_P(PC, PF)                                                                              \
  if (pc == PC && pf == PF) {                                                                        \
    if (wide) mg_prolong_kernel<PC, PF, 12><<<grid, block, 0, s>>>(m, coarse, Q, fine, ncol);        \
    else mg_prolong_kernel<PC, PF, 4><<<grid, block, 0, s>>>(m, coarse, Q, fine, ncol);              \
    return hipGetLastError() == hipSuccess ? 0 : -2;                                                 \
  }
  LQ_MG_P(64, 64)
  LQ_MG_P(64, 32)
  LQ_MG_P(32, 32)
  LQ_MG_P(32, 64)
#undef LQ_MG_P
  return -1;
}

int launch_mg_stencil(const MgGeom& m, int p, const void* M, int d0, int nd, FieldRef in, FieldRef out, FieldRef x,
                      double a, double sgn, int par_out, int ncol, hipStream_t s) {
  if (ncol <= 0) return 0;
  if (2 * m.nv > 64 || d0 < 0 || nd < 0 || d0 + nd > 9 || par_out < 0 || par_out > 2) return -1;
  const bool wide = ncol > 4;
  dim3 grid(par_out == 2 ? m.Vc : m.Vc / 2, wide ? (ncol + 11) / 12 : 1), block(64);
  if (p == 64 && wide && mg_use_mfma())
    mg_stencil_mfma_kernel<64><<<grid, dim3(64 * ((2 * m.nv + 15) / 16)), 0, s>>>(m, M, d0, nd, in, out, x, a, sgn,
                                                                               par_out, ncol);
  else if (p == 64 && wide) mg_stencil_kernel<64, 12><<<grid, block, 0, s>>>(m, M, d0, nd, in, out, x, a, sgn, par_out, ncol);
  else if (p == 64) mg_stencil_kernel<64, 4><<<grid, block, 0, s>>>(m, M, d0, nd, in, out, x, a, sgn, par_out, ncol);
  else if (p == 32 && wide && mg_use_mfma())
    mg_stencil_mfma_kernel<32><<<grid, dim3(64 * ((2 * m.nv + 15) / 16)), 0, s>>>(m, M, d0, nd, in, out, x, a, sgn,
                                                                               par_out, ncol);
  else if (p == 32 && wide) mg_stencil_kernel<32, 12><<<grid, block, 0, s>>>(m, M, d0, nd, in, out, x, a, sgn, par_out, ncol);
  else if (p == 32) mg_stencil_kernel<32, 4><<<grid, block, 0, s>>>(m, M, d0, nd, in, out, x, a, sgn, par_out, ncol);
  else return -1;
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_site_inverse(const MgGeom& m, const void* Dc64, void* Ahat64, void* work, int* bad, hipStream_t s) {
  mg_site_inverse_kernel<<<m.Vc, 64, 0, s>>>(m, (const double2*)Dc64, (double2*)Ahat64, (double2*)work, bad);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_site_mul(const MgGeom& m, const void* Dc64, void* Ahat64, hipStream_t s) {
  mg_site_mul_kernel<<<dim3(m.Vc, 8), 64, 0, s>>>(m, (const double2*)Dc64, (double2*)Ahat64);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_gather(const MgGeom& m, FieldRef fine, void* Q64, hipStream_t s) {
  const int64_t n = (int64_t)m.Vc * m.B * 2 * m.nv;
  mg_gather_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(m, fine, (double2*)Q64);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_orth(const MgGeom& m, void* Q64, int* bad, hipStream_t s) {
  mg_orth_kernel<<<m.Vc * 2, 256, 0, s>>>(m, (double2*)Q64, bad);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_probe_restrict(const MgGeom& m, const void* Q64, FieldRef fine, int ncol, int k0, int cls, void* Dc64,
                             hipStream_t s) {
  if (ncol <= 0) return 0;
  if (2 * m.nv > 64 || ncol > 12) return -1;
  mg_probe_restrict_kernel<<<m.Vc, 256, 0, s>>>(m, (const double2*)Q64, fine, ncol, k0, cls, (double2*)Dc64);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_probe_fine(const MgGeom& m, const void* Q64, FieldRef fine, int ncol, int k0, int cls, hipStream_t s) {
  const int64_t n = (int64_t)m.Vc * m.B * ncol;
  if (n <= 0) return 0;
  mg_probe_fine_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(m, (const double2*)Q64, fine, ncol, k0, cls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_narrow(const void* src64, void* dst32, int64_t n_complex, hipStream_t s) {
  if (n_complex <= 0) return 0;
  mg_narrow_kernel<<<grid_for(n_complex, 256), 256, 0, s>>>((const double2*)src64, (float2*)dst32, n_complex);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_random(FieldRef fine, int ncol, uint64_t seed, hipStream_t s) {
  const int64_t n = (int64_t)ncol * 2 * fine.Vh;
  if (n <= 0) return 0;
  mg_random_kernel<<<grid_for(n, 256), 256, 0, s>>>(fine, ncol, seed);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_mg_cgs(int prec, const FieldRef* W, const FieldRef* Z, int k, FieldRef w, FieldRef z, int ncol, int npar,
                  int gridx, double* partial, double* coef, hipStream_t s) {
  if (k <= 0 || ncol <= 0) return 0;
  if (k > 8 || (prec != 32 && prec != 64)) return -1;
  MgVecSet Ws{}, Zs{};
  for (int j = 0; j < k; ++j) {
    Ws.f[j] = W[j];
    Zs.f[j] = Z[j];
  }
  dim3 grid(gridx, ncol);
  if (prec == 32) mg_mdot_kernel<32><<<grid, 256, 0, s>>>(Ws, k, w, npar, partial);
  else mg_mdot_kernel<64><<<grid, 256, 0, s>>>(Ws, k, w, npar, partial);
  mg_mdot_sum_kernel<<<(k * ncol + 63) / 64, 64, 0, s>>>(partial, k, ncol, gridx, coef);
  if (prec == 32) mg_maxmy_kernel<32><<<grid, 256, 0, s>>>(Ws, Zs, k, w, z, npar, coef);
  else mg_maxmy_kernel<64><<<grid, 256, 0, s>>>(Ws, Zs, k, w, z, npar, coef);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace lq
