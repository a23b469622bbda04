// Ingest and pack (canonical FP64 AoS <-> even-odd SoA in FP64/FP32/FP16),
// precision conversion, and small utility kernels.
//
// Canonical host layout: site s = x + Lx*(y + Ly*(z + Lz*t)); gauge links
// [V][4][3][3] complex128 (U_mu(x)[row][col], link x -> x+mu); fields
// [col][V][NC] complex128.  Device layouts are described in lq_common.h.
#include <cstring>

#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

__device__ __forceinline__ void site_coords(int64_t s, const Geom& g, int c[4]) {
  c[0] = (int)(s % g.L[0]);
  s /= g.L[0];
  c[1] = (int)(s % g.L[1]);
  s /= g.L[1];
  c[2] = (int)(s % g.L[2]);
  c[3] = (int)(s / g.L[2]);
}

__device__ __forceinline__ int64_t coords_site(const int c[4], const Geom& g) {
  return c[0] + (int64_t)g.L[0] * (c[1] + (int64_t)g.L[1] * (c[2] + (int64_t)g.L[2] * c[3]));
}

// One thread per (site, mu).  hisq_hop = 0: plain copy; 1 or 3: multiply by
// 1/2 eta_mu(x) (MILC phases) and by -1 when a hop of that length from x along
// +t crosses the antiperiodic time boundary.  Values are divided by `scale`.
template <int P>
__global__ void pack_links_kernel(Geom g, const double2* aos, void* out, int ne, int hisq_hop, double inv_scale) {
  const int64_t V = 2 * (int64_t)g.Vh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * 4) return;
  const int mu = (int)(i & 3);
  const int64_t s = i >> 2;
  int c[4];
  site_coords(s, g, c);
  const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
  const int cb = (int)(s >> 1);
  double f = inv_scale;
  if (hisq_hop) {
    int eta;
    if (mu == 0) eta = c[3];
    else if (mu == 1) eta = c[3] + c[0];
    else if (mu == 2) eta = c[3] + c[0] + c[1];
    else eta = 0;
    f *= (eta & 1) ? -0.5 : 0.5;
    if (mu == 3 && g.ap && c[3] + hisq_hop >= g.L[3]) f = -f;
  }
  const double2* src = aos + (s * 4 + mu) * 9;
  for (int e = 0; e < ne; ++e) {
    double2 d = src[e];
    d.x *= f;
    d.y *= f;
    const int64_t o = tix(par * 4 + mu, e, ne, cb, g.Vh);
    if constexpr (P == 64) ((double2*)out)[o] = d;
    else if constexpr (P == 32) ((float2*)out)[o] = make_float2((float)d.x, (float)d.y);
    else ((unsigned*)out)[o] = (unsigned)f2h((float)d.x) | ((unsigned)f2h((float)d.y) << 16);
  }
}

int launch_pack_links(const Geom& g, const double* aos, void* out, int prec, int ne, int hisq_hop, double scale,
                      hipStream_t s) {
  const int64_t n = 2 * (int64_t)g.Vh * 4;
  const int bs = 256;
  const int nb = (int)((n + bs - 1) / bs);
  const double inv = 1.0 / scale;
  if (prec == 64) pack_links_kernel<64><<<nb, bs, 0, s>>>(g, (const double2*)aos, out, ne, hisq_hop, inv);
  else if (prec == 32) pack_links_kernel<32><<<nb, bs, 0, s>>>(g, (const double2*)aos, out, ne, hisq_hop, inv);
  else pack_links_kernel<16><<<nb, bs, 0, s>>>(g, (const double2*)aos, out, ne, hisq_hop, inv);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// max |re|,|im| over an FP64 array (one value, host-synchronous)
__global__ void maxabs_kernel(const double* a, int64_t n, unsigned long long* out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(a[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

double link_maxabs(const double* aos, int64_t n, hipStream_t s) {
  unsigned long long* d = nullptr;
  if (hipMallocAsync((void**)&d, sizeof(*d), s) != hipSuccess) return -1.0;
  hipMemsetAsync(d, 0, sizeof(*d), s);
  maxabs_kernel<<<1024, 256, 0, s>>>(aos, n, d);
  unsigned long long h = 0;
  hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
  hipStreamSynchronize(s);
  hipFreeAsync(d, s);
  double v;
  std::memcpy(&v, &h, sizeof(v));
  return v;
}

// One thread per (column, parity slot, cb).
template <int P, int NC>
__global__ void pack_field_kernel(Geom g, const double2* aos, int ncol, FieldRef out, int par_sel) {
  const int npar = par_sel == 2 ? 2 : 1;
  const int64_t nslot = (int64_t)ncol * npar * g.Vh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslot) return;
  const int cb = (int)(i % g.Vh);
  const int64_t r = i / g.Vh;
  const int col = (int)(r / npar);
  const int par = par_sel == 2 ? (int)(r % npar) : par_sel;
  int c[4];
  cb_coords(cb, par, g, c);
  const int64_t s = c[0] + (int64_t)g.L[0] * (c[1] + (int64_t)g.L[1] * (c[2] + (int64_t)g.L[2] * c[3]));
  const int64_t V = 2 * (int64_t)g.Vh;
  using R = typename RealOf<P>::T;
  cx<R> v[NC];
  const double2* src = aos + ((int64_t)col * V + s) * NC;
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = {(R)src[k].x, (R)src[k].y};
  IO<P, NC>::store(out, blk_index(out, col, par), cb, v);
}

template <int P, int NC>
__global__ void unpack_field_kernel(Geom g, FieldRef in, int ncol, double2* aos, int par_sel) {
  const int npar = par_sel == 2 ? 2 : 1;
  const int64_t nslot = (int64_t)ncol * npar * g.Vh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslot) return;
  const int cb = (int)(i % g.Vh);
  const int64_t r = i / g.Vh;
  const int col = (int)(r / npar);
  const int par = par_sel == 2 ? (int)(r % npar) : par_sel;
  int c[4];
  cb_coords(cb, par, g, c);
  const int64_t s = c[0] + (int64_t)g.L[0] * (c[1] + (int64_t)g.L[1] * (c[2] + (int64_t)g.L[2] * c[3]));
  const int64_t V = 2 * (int64_t)g.Vh;
  using R = typename RealOf<P>::T;
  cx<R> v[NC];
  IO<P, NC>::load(in, blk_index(in, col, par), cb, v);
  double2* dst = aos + ((int64_t)col * V + s) * NC;
#pragma unroll
  for (int k = 0; k < NC; ++k) dst[k] = make_double2((double)v[k].re, (double)v[k].im);
}

#define LQ_DISPATCH_PNC(P_, NC_, CALL)              \
  do {                                             \
    if (NC_ == 12) {                               \
      if (P_ == 64) { CALL(64, 12); }              \
      else if (P_ == 32) { CALL(32, 12); }         \
      else { CALL(16, 12); }                       \
    } else {                                       \
      if (P_ == 64) { CALL(64, 3); }               \
      else if (P_ == 32) { CALL(32, 3); }          \
      else { CALL(16, 3); }                        \
    }                                              \
  } while (0)

int launch_pack_field(const Geom& g, const double* aos, int ncol, int nc, FieldRef out, int prec, int par_sel,
                      hipStream_t s) {
  const int npar = par_sel == 2 ? 2 : 1;
  const int64_t n = (int64_t)ncol * npar * g.Vh;
  if (n == 0) return 0;
  const int bs = 256;
  const int nb = (int)((n + bs - 1) / bs);
#define LQ_CALL(PP, NN) pack_field_kernel<PP, NN><<<nb, bs, 0, s>>>(g, (const double2*)aos, ncol, out, par_sel)
  LQ_DISPATCH_PNC(prec, nc, LQ_CALL);
#undef LQ_CALL
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_unpack_field(const Geom& g, FieldRef in, int prec, int ncol, int nc, double* aos, int par_sel,
                        hipStream_t s) {
  const int npar = par_sel == 2 ? 2 : 1;
  const int64_t n = (int64_t)ncol * npar * g.Vh;
  if (n == 0) return 0;
  const int bs = 256;
  const int nb = (int)((n + bs - 1) / bs);
#define LQ_CALL(PP, NN) unpack_field_kernel<PP, NN><<<nb, bs, 0, s>>>(g, in, ncol, (double2*)aos, par_sel)
  LQ_DISPATCH_PNC(prec, nc, LQ_CALL);
#undef LQ_CALL
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// dst(P1) = src(P2), one thread per site slot
template <int P1, int P2, int NC>
__global__ void convert_kernel(FieldRef dst, FieldRef src, int64_t nslot, int Vh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslot) return;
  const int cb = (int)(i % Vh);
  const int64_t blk = i / Vh;
  using R1 = typename RealOf<P1>::T;
  using R2 = typename RealOf<P2>::T;
  cx<R2> v[NC];
  IO<P2, NC>::load(src, blk, cb, v);
  cx<R1> w[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) w[k] = {(R1)v[k].re, (R1)v[k].im};
  IO<P1, NC>::store(dst, blk, cb, w);
}

template <int P1, int P2, int NC>
__global__ void axpy_mixed_kernel(FieldRef y, FieldRef x, int64_t nslot, int Vh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslot) return;
  const int cb = (int)(i % Vh);
  const int64_t blk = i / Vh;
  using R1 = typename RealOf<P1>::T;
  using R2 = typename RealOf<P2>::T;
  cx<R2> v[NC];
  cx<R1> w[NC];
  IO<P2, NC>::load(x, blk, cb, v);
  IO<P1, NC>::load(y, blk, cb, w);
#pragma unroll
  for (int k = 0; k < NC; ++k) w[k] = {w[k].re + (R1)v[k].re, w[k].im + (R1)v[k].im};
  IO<P1, NC>::store(y, blk, cb, w);
}

#define LQ_PAIR_DISPATCH(KERNEL, P1_, P2_, NC_, ...)                                              \
  do {                                                                                             \
    const int key = (P1_) * 1000 + (P2_);                                                          \
    if (NC_ == 12) {                                                                               \
      switch (key) {                                                                               \
        case 64064: KERNEL<64, 64, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 64032: KERNEL<64, 32, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 64016: KERNEL<64, 16, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 32064: KERNEL<32, 64, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 32032: KERNEL<32, 32, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 32016: KERNEL<32, 16, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 16064: KERNEL<16, 64, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 16032: KERNEL<16, 32, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        case 16016: KERNEL<16, 16, 12><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                      \
        default: return -1;                                                                        \
      }                                                                                            \
    } else {                                                                                       \
      switch (key) {                                                                               \
        case 64064: KERNEL<64, 64, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 64032: KERNEL<64, 32, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 64016: KERNEL<64, 16, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 32064: KERNEL<32, 64, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 32032: KERNEL<32, 32, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 32016: KERNEL<32, 16, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 16064: KERNEL<16, 64, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 16032: KERNEL<16, 32, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        case 16016: KERNEL<16, 16, 3><<<nb, bs, 0, s>>>(__VA_ARGS__); break;                       \
        default: return -1;                                                                        \
      }                                                                                            \
    }                                                                                              \
  } while (0)

int launch_convert(FieldRef dst, int pdst, FieldRef src, int psrc, int nc, int ncol, int npar, int Vh,
                   hipStream_t s) {
  const int64_t n = (int64_t)ncol * npar * Vh;
  if (n == 0) return 0;
  const int bs = 256;
  const int nb = (int)((n + bs - 1) / bs);
  LQ_PAIR_DISPATCH(convert_kernel, pdst, psrc, nc, dst, src, n, Vh);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_axpy_mixed(FieldRef y, int py, FieldRef x, int px, int nc, int ncol, int npar, int Vh, hipStream_t s) {
  const int64_t n = (int64_t)ncol * npar * Vh;
  if (n == 0) return 0;
  const int bs = 256;
  const int nb = (int)((n + bs - 1) / bs);
  LQ_PAIR_DISPATCH(axpy_mixed_kernel, py, px, nc, y, x, n, Vh);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

__global__ void fill_zero_kernel(uint4* p, int64_t n16, unsigned char* tail, int ntail) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
  if (i < ntail) tail[i] = 0;
}

int launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return 0;
  const int64_t n16 = (int64_t)(bytes / 16);
  const int ntail = (int)(bytes % 16);
  const int64_t n = n16 > ntail ? n16 : ntail;
  const int bs = 256;
  fill_zero_kernel<<<(int)((n + bs - 1) / bs), bs, 0, s>>>((uint4*)p, n16, (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

__global__ void swap_bytes_kernel(uint4* a, uint4* b, int64_t n16, unsigned char* ta, unsigned char* tb, int ntail) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) {
    const uint4 x = a[i], y = b[i];
    a[i] = y;
    b[i] = x;
  }
  if (i < ntail) {
    const unsigned char x = ta[i], y = tb[i];
    ta[i] = y;
    tb[i] = x;
  }
}

int launch_swap_bytes(void* a, void* b, size_t bytes, hipStream_t s) {
  if (bytes == 0 || a == b) return 0;
  const int64_t n16 = (int64_t)(bytes / 16);
  const int ntail = (int)(bytes % 16);
  const int64_t n = n16 > ntail ? n16 : ntail;
  const int bs = 256;
  swap_bytes_kernel<<<(int)((n + bs - 1) / bs), bs, 0, s>>>((uint4*)a, (uint4*)b, n16,
                                                            (unsigned char*)a + n16 * 16,
                                                            (unsigned char*)b + n16 * 16, ntail);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq

namespace lq {

// Calibration copy: one 16-byte chunk per lane, read once and written once.
__global__ void __launch_bounds__(256) stream_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

int launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return 0;
  stream_copy_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>((const uint4*)src, (uint4*)dst, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq
