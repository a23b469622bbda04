// Vector kernels of the Krylov solvers: fused axpy-family updates, per-column
// FP64 reductions and the scalar recurrences (CG, BiCGStab, multi-shift CG),
// all with device-resident per-column scalars so that the host only polls
// residual norms.
//
// Reductions are deterministic: a fixed grid (set by the volume only, not by
// the number of columns) writes per-block partials reduced in a fixed order
// (wave butterfly, then waves in index order); the scalar kernels sum the
// partials of a column in block order.  A column's result therefore does not
// depend on which other columns share the batch.
#include "lq_common.h"
#include "lq_kernels.h"

namespace lq {

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* out) {
  __shared__ double sm[NV][16];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sm[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += sm[k][i];
      out[k] = s;
    }
  }
}

template <typename R, int NC>
__device__ __forceinline__ void dot_acc(const cx<R>* a, const cx<R>* b, double& re, double& im) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    re += (double)a[k].re * (double)b[k].re + (double)a[k].im * (double)b[k].im;
    im += (double)a[k].re * (double)b[k].im - (double)a[k].im * (double)b[k].re;
  }
}
template <typename R, int NC>
__device__ __forceinline__ double norm_acc(const cx<R>* a) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) s += (double)a[k].re * (double)a[k].re + (double)a[k].im * (double)a[k].im;
  return s;
}

constexpr bool op_reduces(int op) {
  return op == OP_CG || op == OP_BICG_XR || op == OP_DOT || op == OP_NORM2 || op == OP_DOT_NORM ||
         op == OP_XMY_NORM;
}

template <int P, int NC, int OP>
__global__ void __launch_bounds__(256) blas_kernel(BlasArgs A) {
  using R = typename RealOf<P>::T;
  using IOt = IO<P, NC>;
  const int col = blockIdx.y;
  const int64_t n = (int64_t)A.npar * A.Vh;
  cx<R> c0 = {0, 0}, c1 = {0, 0};
  if (A.st) {
    const double* s = A.st + (int64_t)col * ST_STRIDE;
    c0 = {(R)s[A.c0], (R)s[A.c0 + 1]};
    c1 = {(R)s[A.c1], (R)s[A.c1 + 1]};
  } else {
    c0 = {(R)A.imm[0], (R)A.imm[1]};
    c1 = {(R)A.imm[2], (R)A.imm[3]};
  }
  double red[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int par = (int)(j / A.Vh);
    const int cb = (int)(j - (int64_t)par * A.Vh);
    const int64_t blk = (int64_t)col * A.npar + par;
    cx<R> a[NC], b[NC];
    if constexpr (OP == OP_AXPY || OP == OP_AXMY) {
      IOt::load(A.f[0], blk, cb, a);
      IOt::load(A.f[1], blk, cb, b);
#pragma unroll
      for (int k = 0; k < NC; ++k) b[k] = OP == OP_AXPY ? b[k] + c0 * a[k] : b[k] - c0 * a[k];
      IOt::store(A.f[1], blk, cb, b);
    } else if constexpr (OP == OP_XPAY) {
      IOt::load(A.f[0], blk, cb, a);
      IOt::load(A.f[1], blk, cb, b);
#pragma unroll
      for (int k = 0; k < NC; ++k) b[k] = a[k] + c0 * b[k];
      IOt::store(A.f[1], blk, cb, b);
    } else if constexpr (OP == OP_CG) {
      cx<R> x[NC];
      IOt::load(A.f[0], blk, cb, a);  // p
      IOt::load(A.f[2], blk, cb, x);
#pragma unroll
      for (int k = 0; k < NC; ++k) x[k] = x[k] + c0 * a[k];
      IOt::store(A.f[2], blk, cb, x);
      IOt::load(A.f[1], blk, cb, a);  // q
      IOt::load(A.f[3], blk, cb, b);  // r
#pragma unroll
      for (int k = 0; k < NC; ++k) b[k] = b[k] - c0 * a[k];
      IOt::store(A.f[3], blk, cb, b);
      IOt::load(A.f[3], blk, cb, b);  // reduce what was stored (rounded)
      red[0] += norm_acc<R, NC>(b);
    } else if constexpr (OP == OP_BICG_XR) {
      cx<R> x[NC], s[NC];
      IOt::load(A.f[0], blk, cb, a);  // p
      IOt::load(A.f[1], blk, cb, s);  // s
      IOt::load(A.f[3], blk, cb, x);
#pragma unroll
      for (int k = 0; k < NC; ++k) x[k] = x[k] + c0 * a[k] + c1 * s[k];
      IOt::store(A.f[3], blk, cb, x);
      IOt::load(A.f[2], blk, cb, a);  // t
#pragma unroll
      for (int k = 0; k < NC; ++k) s[k] = s[k] - c1 * a[k];
      IOt::store(A.f[1], blk, cb, s);
      IOt::load(A.f[1], blk, cb, s);
      IOt::load(A.f[4], blk, cb, b);  // rhat
      dot_acc<R, NC>(b, s, red[0], red[1]);
      red[2] += norm_acc<R, NC>(s);
    } else if constexpr (OP == OP_BICG_P) {
      cx<R> p[NC];
      IOt::load(A.f[0], blk, cb, a);  // r
      IOt::load(A.f[1], blk, cb, b);  // v
      IOt::load(A.f[2], blk, cb, p);
#pragma unroll
      for (int k = 0; k < NC; ++k) p[k] = a[k] + c0 * (p[k] - c1 * b[k]);
      IOt::store(A.f[2], blk, cb, p);
    } else if constexpr (OP == OP_DOT || OP == OP_DOT_NORM) {
      IOt::load(A.f[0], blk, cb, a);
      IOt::load(A.f[1], blk, cb, b);
      dot_acc<R, NC>(a, b, red[0], red[1]);
      if constexpr (OP == OP_DOT_NORM) red[2] += norm_acc<R, NC>(a);
    } else if constexpr (OP == OP_NORM2) {
      IOt::load(A.f[0], blk, cb, a);
      red[0] += norm_acc<R, NC>(a);
    } else if constexpr (OP == OP_XMY_NORM) {
      IOt::load(A.f[0], blk, cb, a);
      IOt::load(A.f[1], blk, cb, b);
#pragma unroll
      for (int k = 0; k < NC; ++k) b[k] = a[k] - b[k];
      IOt::store(A.f[1], blk, cb, b);
      red[0] += norm_acc<R, NC>(b);
    } else if constexpr (OP == OP_ZERO) {
#pragma unroll
      for (int k = 0; k < NC; ++k) a[k] = {0, 0};
      IOt::store(A.f[0], blk, cb, a);
    } else if constexpr (OP == OP_SCALE) {
      IOt::load(A.f[0], blk, cb, a);
#pragma unroll
      for (int k = 0; k < NC; ++k) a[k] = c0 * a[k];
      IOt::store(A.f[0], blk, cb, a);
    } else if constexpr (OP == OP_G5) {
      IOt::load(A.f[0], blk, cb, a);
#pragma unroll
      for (int k = NC / 2; k < NC; ++k) a[k] = -a[k];
      IOt::store(A.f[1], blk, cb, a);
    } else if constexpr (OP == OP_LC_G5) {
      IOt::load(A.f[0], blk, cb, a);
      IOt::load(A.f[1], blk, cb, b);
#pragma unroll
      for (int k = 0; k < NC; ++k) a[k] = c0 * a[k] + (k < NC / 2 ? c1 * b[k] : -(c1 * b[k]));
      IOt::store(A.f[2], blk, cb, a);
    } else if constexpr (OP == OP_COPY) {
      IOt::load(A.f[0], blk, cb, a);
      IOt::store(A.f[1], blk, cb, a);
    } else if constexpr (OP == OP_PLC) {
      // upper spins see g5 = +1, lower spins g5 = -1
      const double* q = A.pcol + (int64_t)col * 4;
      const R p0 = (R)q[0], pu = (R)(q[1] * (q[2] + q[3])), pl = (R)(q[1] * (q[2] - q[3]));
      IOt::load(A.f[0], blk, cb, a);
      IOt::load(A.f[1], blk, cb, b);
#pragma unroll
      for (int k = 0; k < NC; ++k) a[k] = p0 * a[k] + (k < NC / 2 ? pu : pl) * b[k];
      IOt::store(A.f[2], blk, cb, a);
    }
  }
  if constexpr (op_reduces(OP)) {
    block_reduce_store<4>(red, A.partial + ((int64_t)col * gridDim.x + blockIdx.x) * 4);
  }
}

int blas_gridx(int64_t nsite) {
  int64_t g = (nsite + 255) / 256;
  if (g > 512) g = 512;
  if (g < 1) g = 1;
  return (int)g;
}

template <int P, int NC>
static void blas_dispatch(const BlasArgs& A, dim3 grid, dim3 block, hipStream_t s) {
#define LQ_OPC(OPX) \
  case OPX: blas_kernel<P, NC, OPX><<<grid, block, 0, s>>>(A); break;
  switch (A.op) {
    LQ_OPC(OP_AXPY) LQ_OPC(OP_AXMY) LQ_OPC(OP_XPAY) LQ_OPC(OP_CG) LQ_OPC(OP_BICG_XR) LQ_OPC(OP_BICG_P)
    LQ_OPC(OP_DOT) LQ_OPC(OP_NORM2) LQ_OPC(OP_DOT_NORM) LQ_OPC(OP_XMY_NORM) LQ_OPC(OP_ZERO) LQ_OPC(OP_SCALE)
    LQ_OPC(OP_G5) LQ_OPC(OP_LC_G5) LQ_OPC(OP_COPY) LQ_OPC(OP_PLC)
    default: break;
  }
#undef LQ_OPC
}

int launch_blas(const BlasArgs& A, hipStream_t s) {
  if (A.ncol == 0) return 0;
  dim3 grid(A.gridx, A.ncol), block(256);
  if (A.nc == 12) {
    if (A.prec == 64) blas_dispatch<64, 12>(A, grid, block, s);
    else if (A.prec == 32) blas_dispatch<32, 12>(A, grid, block, s);
    else blas_dispatch<16, 12>(A, grid, block, s);
  } else {
    if (A.prec == 64) blas_dispatch<64, 3>(A, grid, block, s);
    else if (A.prec == 32) blas_dispatch<32, 3>(A, grid, block, s);
    else blas_dispatch<16, 3>(A, grid, block, s);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ------------------------------------------------------------ scalars
// The scalar kernels run one workgroup of kScalarThreads per column; every
// thread executes the same code and ends with the same values.  The partials
// of a column are summed thread-strided in a fixed order, then by a wave
// butterfly and a fixed-order sum over the waves, so the result is bitwise
// identical in every thread and independent of timing and of the batch.
constexpr int kScalarThreads = 256;
__device__ __forceinline__ double sum_r(const double* p, int gridx, int k) {
  __shared__ double wsum[kScalarThreads / 64];
  double s = 0;
  for (int b = (int)threadIdx.x; b < gridx; b += kScalarThreads) s += p[b * 4 + k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < kScalarThreads / 64; ++w) t += wsum[w];
  __syncthreads();  // wsum is reused by the next sum
  return t;
}
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ bool finite_c(cx<double> a) { return isfinite(a.re) && isfinite(a.im); }

__global__ void scalar_kernel(int op, const double* partial, int gridx, int ncol, double* st) {
  const int col = blockIdx.x;
  if (col >= ncol) return;
  double* s = st + (int64_t)col * ST_STRIDE;
  const double* p = partial + (int64_t)col * gridx * 4;
  // the three partial sums every operation draws on, by the whole workgroup;
  // then one wave reads and updates the state (lanes in lockstep, so every
  // read precedes every write)
  const double r0 = sum_r(p, gridx, 0), r1 = sum_r(p, gridx, 1), r2 = sum_r(p, gridx, 2);
  if (threadIdx.x >= 64) return;
  const cx<double> c01 = {r0, r1};
  const bool active = s[ST_ACTIVE] != 0.0;
  auto setc = [&](int off, cx<double> v) { s[off] = v.re; s[off + 1] = v.im; };
  auto getc = [&](int off) { return cx<double>{s[off], s[off + 1]}; };
  switch (op) {
    case SC_CG_ALPHA: {
      // <p, A p> <= 0 can only come from rounding in low-precision storage
      // (A is positive definite): flag a restart of the column (flag 1) and
      // take no step; a non-finite value is a numeric error (flag 2)
      const double pap = r0;
      double a = s[ST_RR] / pap;
      if (!isfinite(pap)) {
        s[ST_FLAG] = 2;
        a = 0;
      } else if (!(pap > 0.0) || !isfinite(a)) {
        if (active) s[ST_FLAG] = 1;
        a = 0;
      }
      setc(ST_ALPHA, {active ? a : 0.0, 0.0});
      break;
    }
    case SC_CG_BETA: {
      const double rr = r0;
      double b = rr / s[ST_RR];
      if (!isfinite(rr)) s[ST_FLAG] = 2;
      if (!isfinite(b)) b = 0;
      if (s[ST_FLAG] == 1) {
        // the column took no step (SC_CG_ALPHA lost positivity): restart its
        // direction with p = r, here on the device, so that iterations whose
        // state the host does not read restart as well
        b = 0;
        s[ST_FLAG] = 0;
        s[ST_NRST] += 1;
      }
      setc(ST_BETA, {active ? b : 0.0, 0.0});
      s[ST_RR] = rr;
      break;
    }
    case SC_BICG_ALPHA: {
      const cx<double> d = c01;
      cx<double> a = cdiv(getc(ST_RHO), d);
      if (!finite_c(a) || (d.re == 0 && d.im == 0)) { s[ST_FLAG] = 1; a = {0, 0}; }
      setc(ST_ALPHA, active ? a : cx<double>{0, 0});
      break;
    }
    case SC_BICG_OMEGA: {
      const cx<double> ts = c01;
      const double tt = r2;
      cx<double> w = {ts.re / tt, ts.im / tt};
      if (!finite_c(w) || tt == 0.0) { s[ST_FLAG] = 1; w = {0, 0}; }
      setc(ST_OMEGA, active ? w : cx<double>{0, 0});
      break;
    }
    case SC_BICG_BETA: {
      const cx<double> rho = c01;
      const double rr = r2;
      cx<double> b = cdiv(rho, getc(ST_RHO)) * cdiv(getc(ST_ALPHA), getc(ST_OMEGA));
      if (!finite_c(b)) { b = {0, 0}; if (active) s[ST_FLAG] = 1; }
      if (!isfinite(rr)) s[ST_FLAG] = 2;
      setc(ST_BETA, active ? b : cx<double>{0, 0});
      setc(ST_RHO, rho);
      s[ST_RR] = rr;
      break;
    }
    case SC_SET_RR:
      s[ST_RR] = r0;
      if (!isfinite(s[ST_RR])) s[ST_FLAG] = 2;
      break;
    case SC_SET_RHO_RR: {
      const cx<double> d = c01;
      setc(ST_RHO, conj(d));
      s[ST_RR] = r2;
      break;
    }
    case SC_DOT_TO_AUX:
      setc(ST_AUX, c01);
      break;
  }
}

int launch_scalar(int op, const double* partial, int gridx, int ncol, double* st, hipStream_t s) {
  if (ncol == 0) return 0;
  scalar_kernel<<<ncol, kScalarThreads, 0, s>>>(op, partial, gridx, ncol, st);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ------------------------------------------------------------ multi-shift CG
// shift state [i][j][8]: 0 zeta, 1 zeta_old, 2 alpha_i, 3 beta_i, 4 active, 5 zeta_new
// One iteration: ms_xr (r -= alpha A p and |r|^2, base columns only), the
// beta step, then ms_p (x_i += alpha_i p_i and p_i = zeta_i r + beta_i p_i,
// every shift: one pass over p_i serves both updates).
// base state (per rhs j): ST_ALPHA, ST_BETA, ST_RR, ST_AUX = alpha_old, ST_AUX+1 = beta_old, ST_RR0 = |b|^2,
// ST_PAD = tol^2 of the multi-shift stage
enum { MS_Z = 0, MS_ZO, MS_A, MS_B, MS_ACT, MS_ZN };

template <int P, int NC>
__global__ void __launch_bounds__(256) ms_xr_kernel(MsArgs A) {
  using R = typename RealOf<P>::T;
  using IOt = IO<P, NC>;
  const int j = blockIdx.y;
  const int64_t n = (int64_t)A.npar * A.Vh;
  const R a = (R)A.st[(int64_t)j * ST_STRIDE + ST_ALPHA];
  double red[1] = {0.0};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int par = (int)(t / A.Vh);
    const int cb = (int)(t - (int64_t)par * A.Vh);
    cx<R> r[NC], q[NC];
    const int64_t bj = (int64_t)j * A.npar + par;
    IOt::load(A.r, bj, cb, r);
    IOt::load(A.ap, bj, cb, q);
#pragma unroll
    for (int k = 0; k < NC; ++k) r[k] = r[k] - a * q[k];
    IOt::store(A.r, bj, cb, r);
    IOt::load(A.r, bj, cb, r);
    red[0] += norm_acc<R, NC>(r);
  }
  block_reduce_store<1>(red, A.partial + ((int64_t)j * gridDim.x + blockIdx.x) * 4);
}

template <int P, int NC>
__global__ void __launch_bounds__(256) ms_p_kernel(MsArgs A) {
  using R = typename RealOf<P>::T;
  using IOt = IO<P, NC>;
  const int j = blockIdx.y;
  const int64_t n = (int64_t)A.npar * A.Vh;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int par = (int)(t / A.Vh);
    const int cb = (int)(t - (int64_t)par * A.Vh);
    cx<R> r[NC];
    IOt::load(A.r, (int64_t)j * A.npar + par, cb, r);
    for (int i = 0; i < A.nshift; ++i) {
      const double* sh = A.sh + ((int64_t)i * A.nrhs + j) * 8;
      // alpha_i is zero for shifts inactive at this iteration's alpha step; a
      // shift retired by this iteration's beta step still takes its x step
      const bool xs = sh[MS_A] != 0.0, ps = sh[MS_ACT] != 0.0;
      if (!xs && !ps) continue;
      const R ai = (R)sh[MS_A], z = (R)sh[MS_Z], b = (R)sh[MS_B];
      const int64_t bi = ((int64_t)i * A.nrhs + j) * A.npar + par;
      cx<R> p[NC];
      IOt::load(A.p, bi, cb, p);
      if (xs) {
        cx<R> x[NC];
        IOt::load(A.x, bi, cb, x);
#pragma unroll
        for (int k = 0; k < NC; ++k) x[k] = x[k] + ai * p[k];
        IOt::store(A.x, bi, cb, x);
      }
      if (ps) {
#pragma unroll
        for (int k = 0; k < NC; ++k) p[k] = z * r[k] + b * p[k];
        IOt::store(A.p, bi, cb, p);
      }
    }
  }
}

// alpha = rr / <p0, A p0>; per shift: zeta_new and alpha_i (shift 0 keeps zeta = 1)
__global__ void ms_alpha_kernel(MsArgs A, const double* sigma) {
  const int j = blockIdx.x;
  if (j >= A.nrhs) return;
  double* s = A.st + (int64_t)j * ST_STRIDE;
  const double pap = sum_r(A.partial + (int64_t)j * A.gridx * 4, A.gridx, 0);
  if (threadIdx.x >= 64) return;  // one wave updates the state (reads before writes)
  double a = s[ST_RR] / pap;
  if (!isfinite(pap)) {
    a = 0;
    s[ST_FLAG] = 2;
  } else if (!(pap > 0.0) || !isfinite(a)) {
    // loss of positivity from low-precision rounding: stop the multi-shift
    // stage for this right-hand side (its iterate stays a valid starting
    // guess for the per-shift refinement)
    a = 0;
    s[ST_FLAG] = 1;
    for (int i = 0; i < A.nshift; ++i) A.sh[((int64_t)i * A.nrhs + j) * 8 + MS_ACT] = 0.0;
  }
  const bool base_active = A.sh[(int64_t)j * 8 + MS_ACT] != 0.0;
  if (!base_active) a = 0.0;
  s[ST_ALPHA] = a;
  const double ao = s[ST_AUX], bo = s[ST_AUX + 1];
  for (int i = 0; i < A.nshift; ++i) {
    double* sh = A.sh + ((int64_t)i * A.nrhs + j) * 8;
    if (i == 0) { sh[MS_ZN] = 1.0; sh[MS_A] = a; continue; }
    const double z = sh[MS_Z], zo = sh[MS_ZO];
    const double den = a * bo * (zo - z) + zo * ao * (1.0 + sigma[i] * a);
    double zn = z * zo * ao / den;
    if (!isfinite(zn) || a == 0.0) zn = z;
    sh[MS_ZN] = zn;
    sh[MS_A] = (sh[MS_ACT] != 0.0 && a != 0.0) ? a * zn / z : 0.0;
  }
}

// beta = rr_new / rr; beta_i = beta (zeta_new/zeta)^2; rotate zeta; retire shifts
__global__ void ms_beta_kernel(MsArgs A) {
  const int j = blockIdx.x;
  if (j >= A.nrhs) return;
  double* s = A.st + (int64_t)j * ST_STRIDE;
  const double rr = sum_r(A.partial + (int64_t)j * A.gridx * 4, A.gridx, 0);
  if (threadIdx.x >= 64) return;  // one wave updates the state (reads before writes)
  double b = rr / s[ST_RR];
  if (!isfinite(b)) b = 0.0;
  if (!isfinite(rr)) s[ST_FLAG] = 2;
  const double tol2 = s[ST_PAD] * s[ST_RR0];
  for (int i = 0; i < A.nshift; ++i) {
    double* sh = A.sh + ((int64_t)i * A.nrhs + j) * 8;
    const double z = sh[MS_Z], zn = sh[MS_ZN];
    sh[MS_B] = (i == 0) ? b : b * (zn / z) * (zn / z);
    sh[MS_ZO] = z;
    sh[MS_Z] = zn;
    // residual of shift i is zeta_i * r
    if (sh[MS_ACT] != 0.0 && zn * zn * rr < tol2) sh[MS_ACT] = (i == 0) ? sh[MS_ACT] : 0.0;
  }
  // the base shift stays active until every shift has converged
  bool any = false;
  for (int i = 1; i < A.nshift; ++i) any |= A.sh[((int64_t)i * A.nrhs + j) * 8 + MS_ACT] != 0.0;
  if (rr < tol2 && !any) A.sh[(int64_t)j * 8 + MS_ACT] = 0.0;
  s[ST_AUX] = s[ST_ALPHA];
  s[ST_AUX + 1] = b;
  s[ST_BETA] = b;
  s[ST_RR] = rr;
}

__global__ void ms_init_kernel(MsArgs A) {
  const int j = blockIdx.x;
  if (j >= A.nrhs) return;
  double* s = A.st + (int64_t)j * ST_STRIDE;
  const double rr = sum_r(A.partial + (int64_t)j * A.gridx * 4, A.gridx, 0);
  if (threadIdx.x >= 64) return;  // one wave updates the state (reads before writes)
  s[ST_RR] = rr;
  s[ST_RR0] = rr;
  s[ST_AUX] = 1.0;
  s[ST_AUX + 1] = 0.0;
  s[ST_FLAG] = 0.0;
  for (int i = 0; i < A.nshift; ++i) {
    double* sh = A.sh + ((int64_t)i * A.nrhs + j) * 8;
    sh[MS_Z] = sh[MS_ZO] = sh[MS_ZN] = 1.0;
    sh[MS_A] = sh[MS_B] = 0.0;
    sh[MS_ACT] = rr > 0.0 ? 1.0 : 0.0;
  }
}

#define LQ_MS_DISPATCH(KER)                                                               \
  do {                                                                                    \
    dim3 grid(A.gridx, A.nrhs), block(256);                                               \
    if (A.nc == 12) {                                                                     \
      if (A.prec == 64) KER<64, 12><<<grid, block, 0, s>>>(A);                            \
      else if (A.prec == 32) KER<32, 12><<<grid, block, 0, s>>>(A);                       \
      else KER<16, 12><<<grid, block, 0, s>>>(A);                                         \
    } else {                                                                              \
      if (A.prec == 64) KER<64, 3><<<grid, block, 0, s>>>(A);                             \
      else if (A.prec == 32) KER<32, 3><<<grid, block, 0, s>>>(A);                        \
      else KER<16, 3><<<grid, block, 0, s>>>(A);                                          \
    }                                                                                     \
  } while (0)

int launch_ms_xr(const MsArgs& A, hipStream_t s) {
  LQ_MS_DISPATCH(ms_xr_kernel);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
int launch_ms_p(const MsArgs& A, hipStream_t s) {
  LQ_MS_DISPATCH(ms_p_kernel);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
int launch_ms_scalar_alpha(const MsArgs& A, const double* sigma, hipStream_t s) {
  ms_alpha_kernel<<<A.nrhs, kScalarThreads, 0, s>>>(A, sigma);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
int launch_ms_scalar_beta(const MsArgs& A, hipStream_t s) {
  ms_beta_kernel<<<A.nrhs, kScalarThreads, 0, s>>>(A);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
int launch_ms_init(const MsArgs& A, hipStream_t s) {
  ms_init_kernel<<<A.nrhs, kScalarThreads, 0, s>>>(A);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lq
