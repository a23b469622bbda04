// Low modes for the overlap operator (sec. 2.3).
//
// The paper computes the low-lying eigenvectors of H_W = g5 D_W(-rho), treats
// the sign function exactly on them and uses the Chebyshev polynomial only on
// the rest; it finds them with a restarted Arnoldi method applied to a
// Chebyshev polynomial of the operator (the polynomial keeps the eigenvectors
// and spreads the wanted end of the spectrum), diagonalising the Hessenberg
// matrix by QR steps.  It also computes low modes of the chirally projected
// overlap operator to deflate the propagator solve.
//
// Both operators are Hermitian here, so the Arnoldi process reduces to
// Lanczos (the Hessenberg matrix is a real symmetric tridiagonal T) and the
// restart is the implicit one: shifted QR steps on T with the unwanted Ritz
// values as shifts compress the basis onto the wanted invariant subspace
// without leaving the tridiagonal form.  The basis is kept orthogonal by
// classical Gram-Schmidt applied twice against all basis vectors.  The
// tall-skinny products with the basis (V^H w, V c, V Q) are plain complex
// FP64 matrix products and go to rocBLAS; the operators are the library's
// stencils.
//
//  * LQ_EIG_HW: A = T_d(Z(H_W^2)), Z maps [cut, b] onto [-1, 1] (d even, so the
//    eigenvalues of H_W^2 below cut become the largest of A), then a
//    Rayleigh-Ritz step with H_W itself splits the +-lambda pairs.
//  * LQ_EIG_OVERLAP: per chirality s the sector operator
//    H_s = D^dag D on the sector = 2 rho^2 (1 + s P_s eps P_s), as
//    A = sigma_top - H_s (its largest eigenvalues are the smallest of H_s),
//    started from a vector of that chirality (H_s keeps the sector).
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>

#include "lq_internal.h"
#include "solver_util.h"

namespace lq {

using zc = std::complex<double>;

static rocblas_handle rb_handle(lq_ctx* c, hipStream_t s) {
  if (!c->rocblas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    c->rocblas = h;
  }
  rocblas_handle h = (rocblas_handle)c->rocblas;
  rocblas_set_stream(h, s);
  return h;
}

void eig_release(lq_ctx* c) {
  if (c->rocblas) rocblas_destroy_handle((rocblas_handle)c->rocblas);
  c->rocblas = nullptr;
}

// complex elements of one FP64 Wilson-type column with both parities
static int64_t col_len(const Geom& g) { return (int64_t)2 * g.Vh * 12; }
static rocblas_double_complex* colp(const Vec& v, int j) {
  return (rocblas_double_complex*)v.cols(j).data;
}

// ------------------------------------------------------------------ small dense matrices (host)
// Eigenpairs of a real symmetric n x n matrix A (row-major, destroyed) by
// cyclic Jacobi rotations; w descending, V[i * n + k] = component i of vector k.
static void jacobi_sym(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        const double tau = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double kp = a(k, p), kq = a(k, q);
          a(k, p) = c * kp - s * kq;
          a(k, q) = s * kp + c * kq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double pk = a(p, k), qk = a(q, k);
          a(p, k) = c * pk - s * qk;
          a(q, k) = s * pk + c * qk;
        }
        for (int k = 0; k < n; ++k) {
          const double kp = V[(size_t)k * n + p], kq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * kp - s * kq;
          V[(size_t)k * n + q] = s * kp + c * kq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x) > a(y, y); });
  std::vector<double> V2((size_t)n * n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    w[k] = a(idx[k], idx[k]);
    for (int i = 0; i < n; ++i) V2[(size_t)i * n + k] = V[(size_t)i * n + idx[k]];
  }
  V.swap(V2);
}

// The same for a complex Hermitian matrix: each rotation first turns the
// pivot element real by a phase on its column, then rotates as above.
// w ascending by |w| is left to the caller; here w descending.
static void jacobi_herm(std::vector<zc>& A, int n, std::vector<double>& w, std::vector<zc>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> zc& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += std::norm(a(i, j));
        if (i != j) off += std::norm(a(i, j));
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double r = std::abs(a(p, q));
        if (r < 1e-300) continue;
        const zc ph = std::conj(a(p, q)) / r;  // column q times ph makes a(p, q) real and positive
        for (int k = 0; k < n; ++k) a(k, q) *= ph;
        for (int k = 0; k < n; ++k) a(q, k) *= std::conj(ph);
        for (int k = 0; k < n; ++k) V[(size_t)k * n + q] *= ph;
        const double apq = a(p, q).real();
        const double tau = (a(q, q).real() - a(p, p).real()) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const zc kp = a(k, p), kq = a(k, q);
          a(k, p) = c * kp - s * kq;
          a(k, q) = s * kp + c * kq;
        }
        for (int k = 0; k < n; ++k) {
          const zc pk = a(p, k), qk = a(q, k);
          a(p, k) = c * pk - s * qk;
          a(q, k) = s * pk + c * qk;
        }
        for (int k = 0; k < n; ++k) {
          const zc kp = V[(size_t)k * n + p], kq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * kp - s * kq;
          V[(size_t)k * n + q] = s * kp + c * kq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x).real() > a(y, y).real(); });
  std::vector<zc> V2((size_t)n * n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    w[k] = a(idx[k], idx[k]).real();
    for (int i = 0; i < n; ++i) V2[(size_t)i * n + k] = V[(size_t)i * n + idx[k]];
  }
  V.swap(V2);
}

// One shifted QR step on the symmetric tridiagonal T (dense n x n,
// row-major): T - mu = Q R by Givens rotations of neighbouring rows, then
// T <- R Q + mu = Q^T T Q; Qacc <- Qacc Q.  Entries outside the tridiagonal
// band are rounding and are cleared.
static void qr_shift_step(std::vector<double>& T, int n, double mu, std::vector<double>& Qacc, int nq) {
  auto t = [&](int i, int j) -> double& { return T[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i) t(i, i) -= mu;
  std::vector<double> cs(n), sn(n);
  for (int i = 0; i + 1 < n; ++i) {
    const double x = t(i, i), y = t(i + 1, i);
    const double r = std::hypot(x, y);
    const double c = r > 0 ? x / r : 1.0, s = r > 0 ? y / r : 0.0;
    cs[i] = c;
    sn[i] = s;
    for (int k = 0; k < n; ++k) {  // rows i, i+1: G^T
      const double a = t(i, k), b = t(i + 1, k);
      t(i, k) = c * a + s * b;
      t(i + 1, k) = -s * a + c * b;
    }
  }
  for (int i = 0; i + 1 < n; ++i) {  // R Q: columns i, i+1
    const double c = cs[i], s = sn[i];
    for (int k = 0; k < n; ++k) {
      const double a = t(k, i), b = t(k, i + 1);
      t(k, i) = c * a + s * b;
      t(k, i + 1) = -s * a + c * b;
    }
    for (int k = 0; k < nq; ++k) {
      const double a = Qacc[(size_t)k * n + i], b = Qacc[(size_t)k * n + i + 1];
      Qacc[(size_t)k * n + i] = c * a + s * b;
      Qacc[(size_t)k * n + i + 1] = -s * a + c * b;
    }
  }
  for (int i = 0; i < n; ++i) t(i, i) += mu;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (std::abs(i - j) > 1) t(i, j) = 0.0;
  for (int i = 0; i + 1 < n; ++i) t(i, i + 1) = t(i + 1, i) = 0.5 * (t(i, i + 1) + t(i + 1, i));
}

// ------------------------------------------------------------------ implicitly restarted Lanczos
struct IrlOut {
  std::vector<double> theta;  // the nev largest Ritz values of A, descending
  int restarts = 0, applications = 0;
  double worst_est = 0;       // largest residual estimate |beta_m s_m| / |theta| of them
};

// The nev largest eigenpairs of the Hermitian operator A (FP64, one column at
// a time) by Lanczos with a basis of m vectors, implicit restarts keeping k,
// and full reorthogonalisation (CGS2).  V (m + 1 columns) receives the basis;
// on return its first nev columns are the Ritz vectors.  start(v) fills the
// first basis vector (any nonzero vector in the wanted space).
static int irl(lq_ctx* c, const Geom& g, hipStream_t s, const OpFn& A, const std::function<int(Vec&)>& start,
               int nev, int k, int m, double tol, int max_restarts, Vec& V, IrlOut& out) {
  rocblas_handle h = rb_handle(c, s);
  if (!h) return fail(LQ_EDEVICE, "rocBLAS handle");
  const int64_t N = col_len(g);
  Blas bl;
  int e = blas_prepare(c, bl, g, 2, 1, s);
  if (e) return e;
  DBuf dcoef(sizeof(zc) * (m + 1) * 2, s);
  Vec w = make_vec(g, 64, 12, 1, 2, 0, s), W = make_vec(g, 64, 12, k + 1, 2, 0, s);
  if (!dcoef.p || !w.ok() || !W.ok()) return fail(LQ_ENOMEM, "eigensolver buffers");
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0}, mone = {-1.0, 0.0};
  std::vector<zc> hc(m + 1);
  std::vector<double> nn;
  // w -= V_{0..j} (V_{0..j}^H w), twice; returns the coefficient on column j of both passes
  auto cgs2 = [&](Vec& wv, int jn, zc& cj) -> int {
    cj = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      if (rocblas_zgemv(h, rocblas_operation_conjugate_transpose, N, jn, &one, colp(V, 0), N, colp(wv, 0), 1, &zero,
                        (rocblas_double_complex*)dcoef.p, 1) != rocblas_status_success ||
          rocblas_zgemv(h, rocblas_operation_none, N, jn, &mone, colp(V, 0), N, (rocblas_double_complex*)dcoef.p, 1,
                        &one, colp(wv, 0), 1) != rocblas_status_success)
        return fail(LQ_EDEVICE, "rocBLAS gemv");
      if (hipMemcpyAsync(hc.data(), dcoef.p, sizeof(zc) * jn, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(LQ_EDEVICE, "coefficients");
      cj += hc[jn - 1];
    }
    return 0;
  };
  std::vector<double> alpha(m, 0.0), beta(m, 0.0);  // T: diagonal alpha, off-diagonal beta[j] = T[j+1][j]
  {
    Vec v0 = view(V, 0, 1);
    if ((e = start(v0))) return e;
    if ((e = col_norms(bl, v0, nn))) return e;
    if (!(nn[0] > 0)) return fail(LQ_EINVAL, "eigensolver: zero start vector");
    if ((e = bl.opi(OP_SCALE, &v0, nullptr, nullptr, 1.0 / std::sqrt(nn[0])))) return e;
  }
  int kk = 0;  // current basis length
  for (int rs = 0; rs <= max_restarts; ++rs) {
    for (int j = kk; j < m; ++j) {
      Vec vj = view(V, j, 1);
      if ((e = A(w, vj))) return e;
      ++out.applications;
      zc cj;
      if ((e = cgs2(w, j + 1, cj))) return e;
      alpha[j] = cj.real();
      if ((e = col_norms(bl, w, nn))) return e;
      beta[j] = std::sqrt(nn[0]);
      if (!(beta[j] > 0) || !std::isfinite(beta[j])) return fail(LQ_ENUMERIC, "eigensolver: Lanczos breakdown");
      Vec vn = view(V, j + 1, 1);
      if (launch_convert(vn.f, 64, w.f, 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      if ((e = bl.opi(OP_SCALE, &vn, nullptr, nullptr, 1.0 / beta[j]))) return e;
    }
    // Ritz pairs of T_m
    std::vector<double> T((size_t)m * m, 0.0), th, S;
    for (int i = 0; i < m; ++i) {
      T[(size_t)i * m + i] = alpha[i];
      if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = beta[i];
    }
    std::vector<double> Tc = T;
    jacobi_sym(Tc, m, th, S);
    double worst = 0.0;
    for (int i = 0; i < nev; ++i)
      worst = std::max(worst, std::fabs(beta[m - 1] * S[(size_t)(m - 1) * m + i]) / std::max(std::fabs(th[i]), 1e-300));
    out.worst_est = worst;
    out.restarts = rs;
    if (const char* ev = getenv("LQ_VERBOSE"))
      if (*ev && *ev != '0')
        fprintf(stderr, "[lq] eigensolver restart %d: %d operator applications, worst Ritz estimate %.3e\n", rs,
                out.applications, worst);
    if (worst <= tol || rs == max_restarts) {
      // Ritz vectors: V_{0..nev-1} <- V_m S[:, 0:nev]
      std::vector<zc> Sc((size_t)m * nev);
      for (int i = 0; i < m; ++i)
        for (int l = 0; l < nev; ++l) Sc[(size_t)l * m + i] = S[(size_t)i * m + l];  // column-major m x nev
      DBuf dS(sizeof(zc) * Sc.size(), s);
      if (!dS.p) return fail(LQ_ENOMEM, "eigensolver buffers");
      hipMemcpyAsync(dS.p, Sc.data(), sizeof(zc) * Sc.size(), hipMemcpyHostToDevice, s);
      if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, N, nev, m, &one, colp(V, 0), N,
                        (rocblas_double_complex*)dS.p, m, &zero, colp(W, 0), N) != rocblas_status_success)
        return fail(LQ_EDEVICE, "rocBLAS gemm");
      for (int l = 0; l < nev; ++l)
        if (launch_convert(V.cols(l), 64, W.cols(l), 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      out.theta.assign(th.begin(), th.begin() + nev);
      if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "eigensolver");
      return worst <= tol ? 0 : LQ_ENOCONV;
    }
    // implicit restart: shifted QR steps with the m - k unwanted Ritz values
    std::vector<double> Q((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    for (int i = k; i < m; ++i) qr_shift_step(T, m, th[i], Q, m);
    // V_{0..k} <- V_m Q[:, 0:k+1]
    std::vector<zc> Qc((size_t)m * (k + 1));
    for (int i = 0; i < m; ++i)
      for (int l = 0; l <= k; ++l) Qc[(size_t)l * m + i] = Q[(size_t)i * m + l];
    DBuf dQ(sizeof(zc) * Qc.size(), s);
    if (!dQ.p) return fail(LQ_ENOMEM, "eigensolver buffers");
    hipMemcpyAsync(dQ.p, Qc.data(), sizeof(zc) * Qc.size(), hipMemcpyHostToDevice, s);
    if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, N, k + 1, m, &one, colp(V, 0), N,
                      (rocblas_double_complex*)dQ.p, m, &zero, colp(W, 0), N) != rocblas_status_success)
      return fail(LQ_EDEVICE, "rocBLAS gemm");
    // residual of the compressed factorisation: f = T'[k][k-1] (V Q)_k + beta_{m-1} Q[m-1][k-1] v_m
    const double tk = T[(size_t)k * m + k - 1], sk = beta[m - 1] * Q[(size_t)(m - 1) * m + k - 1];
    {
      Vec f = view(w, 0, 1), wk = view(W, k, 1), vm = view(V, m, 1);
      if (launch_convert(f.f, 64, vm.f, 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      if ((e = bl.opi(OP_SCALE, &f, nullptr, nullptr, sk))) return e;
      if ((e = bl.opi(OP_AXPY, &wk, &f, nullptr, tk))) return e;
    }
    for (int l = 0; l < k; ++l)
      if (launch_convert(V.cols(l), 64, W.cols(l), 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
    zc cdrop;
    if ((e = cgs2(w, k, cdrop))) return e;
    if ((e = col_norms(bl, w, nn))) return e;
    for (int i = 0; i < k; ++i) alpha[i] = T[(size_t)i * m + i];
    for (int i = 0; i + 1 < k; ++i) beta[i] = T[(size_t)(i + 1) * m + i];
    beta[k - 1] = std::sqrt(nn[0]);
    if (!(beta[k - 1] > 0)) return fail(LQ_ENUMERIC, "eigensolver: restart breakdown");
    {
      Vec vk = view(V, k, 1);
      if (launch_convert(vk.f, 64, w.f, 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      if ((e = bl.opi(OP_SCALE, &vk, nullptr, nullptr, 1.0 / beta[k - 1]))) return e;
    }
    kk = k;  // the next Lanczos step starts from v_k
  }
  return LQ_ENOCONV;
}

// ------------------------------------------------------------------ operators and public entry
static int random_start(const Geom& g, hipStream_t s, Vec& v, uint64_t seed, int chir) {
  const int64_t n = col_len(g) * 2;
  std::vector<double> hst(n);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd;
  for (auto& x : hst) x = nd(rng);
  DBuf raw(sizeof(double) * n, s);
  if (!raw.p) return fail(LQ_ENOMEM, "start vector");
  hipMemcpyAsync(raw.p, hst.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
  // canonical [V][4][3] order, so chirality is spin 0,1 (+) or 2,3 (-)
  if (chir != 0) {
    for (int64_t site = 0; site < n / 24; ++site)
      for (int sp = 0; sp < 4; ++sp)
        if ((sp < 2) != (chir > 0))
          for (int k = 0; k < 6; ++k) hst[site * 24 + sp * 6 + k] = 0.0;
    hipMemcpyAsync(raw.p, hst.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
  }
  if (launch_pack_field(g, raw.as<double>(), 1, 12, v.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
  return hipStreamSynchronize(s) == hipSuccess ? 0 : fail(LQ_EDEVICE, "start vector");
}

// H_W eigenpairs of the converged subspace U (n columns): Rayleigh-Ritz with
// H_W (M = U^H H_W U diagonalised on the host), then U <- U G; lam sorted by
// |lam| ascending; res = |H_W u - lam u| per vector.
static int rayleigh_ritz(OpEnv& env, Vec& U, int n, std::vector<double>& lam, std::vector<double>& res,
                         const OpFn& Aop) {
  lq_ctx* c = env.ctx;
  const Geom& g = env.f->g;
  hipStream_t s = env.s;
  rocblas_handle h = rb_handle(c, s);
  const int64_t N = col_len(g);
  Vec Uv = view(U, 0, n);
  Vec HU = make_vec(g, 64, 12, n, 2, 0, s), T = make_vec(g, 64, 12, n, 2, 0, s);
  DBuf dM(sizeof(zc) * n * n, s);
  if (!HU.ok() || !T.ok() || !dM.p) return fail(LQ_ENOMEM, "Rayleigh-Ritz buffers");
  int e = Aop(HU, Uv);
  if (e) return e;
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  for (int col = 0; col < n; ++col)  // M = U^H (H U), column by column (see project_out)
    if (rocblas_zgemv(h, rocblas_operation_conjugate_transpose, N, n, &one, colp(Uv, 0), N, colp(HU, col), 1, &zero,
                      (rocblas_double_complex*)dM.p + (size_t)col * n, 1) != rocblas_status_success)
      return fail(LQ_EDEVICE, "rocBLAS gemv");
  std::vector<zc> Mc((size_t)n * n), M((size_t)n * n), G;
  hipMemcpyAsync(Mc.data(), dM.p, sizeof(zc) * n * n, hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "Rayleigh-Ritz");
  for (int i = 0; i < n; ++i)  // column-major -> row-major, Hermitian part
    for (int j = 0; j < n; ++j) M[(size_t)i * n + j] = 0.5 * (Mc[(size_t)j * n + i] + std::conj(Mc[(size_t)i * n + j]));
  std::vector<double> w;
  jacobi_herm(M, n, w, G);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return std::fabs(w[a]) < std::fabs(w[b]); });
  std::vector<zc> Gc((size_t)n * n);
  lam.resize(n);
  for (int l = 0; l < n; ++l) {
    lam[l] = w[idx[l]];
    for (int i = 0; i < n; ++i) Gc[(size_t)l * n + i] = G[(size_t)i * n + idx[l]];
  }
  hipMemcpyAsync(dM.p, Gc.data(), sizeof(zc) * n * n, hipMemcpyHostToDevice, s);
  if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, N, n, n, &one, colp(Uv, 0), N,
                    (rocblas_double_complex*)dM.p, n, &zero, colp(T, 0), N) != rocblas_status_success)
    return fail(LQ_EDEVICE, "rocBLAS gemm");
  if ((e = vec_copy(Uv, T))) return e;
  // residuals
  if ((e = Aop(HU, Uv))) return e;
  State st(n, s);
  if (!st.ok()) return fail(LQ_ENOMEM, "state");
  for (int l = 0; l < n; ++l) {
    for (int k = 0; k < ST_STRIDE; ++k) st.h(l, k) = 0.0;
    st.h(l, ST_AUX) = lam[l];
  }
  if ((e = st.push())) return e;
  Blas bl;
  if ((e = blas_prepare(c, bl, g, 2, n, s))) return e;
  if ((e = bl.op(OP_AXMY, &Uv, &HU, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX))) return e;
  std::vector<double> rr;
  if ((e = col_norms(bl, HU, rr))) return e;
  res.resize(n);
  for (int l = 0; l < n; ++l) res[l] = std::sqrt(rr[l]);
  return 0;
}

int eigs(lq_ctx* c, const lq_action* act, lq_field* f, int which, int nev, double tol, int max_restarts,
         int degree, double cut, double* evals, lq_stats* st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (f->type != 0) return fail(LQ_EINVAL, "eigensolver needs a Wilson gauge field");
  if (nev < 1 || nev > 1000) return fail(LQ_EINVAL, "nev must be in 1..1000");
  if (!(tol > 0)) tol = 1e-10;
  if (max_restarts <= 0) max_restarts = 200;
  const Geom& g = f->g;
  if ((int64_t)3 * nev + 8 > col_len(g) / 4) return fail(LQ_EINVAL, "nev too large for the lattice");
  OpEnv env{c, f, *act, s};
  env.act.n_lowmodes = 0;  // the eigensolver works with the plain operators
  const int k = nev + std::max(2, nev / 2), m = 2 * k + 2;
  Vec V = make_vec(g, 64, 12, m + 1, 2, 0, s);
  if (!V.ok()) return fail(LQ_ENOMEM, "eigensolver basis");
  const double rho = act->rho;
  int e = 0, status = LQ_OK, apps = 0, restarts = 0;
  std::vector<EigSet> sets;
  std::vector<double> all_vals, all_res;
  if (which == LQ_EIG_HW) {
    HwSpectrum sp{};
    if ((e = hw_spectrum(c, act, f, 300, &sp, s))) return e;
    const double lo2 = sp.theta_min - sp.r_min, hi2 = sp.theta_max + sp.r_max;
    const double top = 1.05 * hi2, cc = cut > 0 ? cut : std::max(4.0 * lo2, lo2 + 0.02 * (hi2 - lo2));
    const int d = degree > 0 ? degree + (degree & 1) : 24;
    if (!(cc > lo2 && cc < top)) return fail(LQ_EINVAL, "filter cut outside the spectrum of H_W^2");
    // A v = T_d(Z(H^2)) v, Z = (2 H^2 - (cc + top)) / (top - cc)
    OpFn A = [&](Vec& out, const Vec& in) { return cheb_filter(env, out, in, cc, top, d); };
    IrlOut io;
    const int r = irl(c, g, s, A, [&](Vec& v) { return random_start(g, s, v, 777, 0); }, nev, k, m, tol, max_restarts,
                      V, io);
    if (r && r != LQ_ENOCONV) return r;
    apps = io.applications * d * 2;
    restarts = io.restarts;
    OpFn H = [&](Vec& out, const Vec& in) { return hw_apply(env, 64, out, in); };
    std::vector<double> lam, res;
    if ((e = rayleigh_ritz(env, V, nev, lam, res, H))) return e;
    // every Ritz value of A must come from below the cut (the filter keeps the order there)
    for (double l : lam)
      if (l * l >= cc) return fail(LQ_EINVAL, "eigensolver: filter cut " + std::to_string(cc) +
                                                   " below the wanted eigenvalues of H_W^2; raise it");
    EigSet es;
    es.which = LQ_EIG_HW;
    es.rho = rho;
    es.chir = 0;
    es.vals = lam;
    es.res = res;
    sets.push_back(std::move(es));
    all_vals = lam;
    all_res = res;
    for (double rr : res)
      if (!(rr <= tol * std::max(1.0, std::fabs(lam.back())))) status = LQ_ENOCONV;
  } else if (which == LQ_EIG_OVERLAP) {
    if ((e = overlap_prepare(env))) return e;
    const double top = 4.0 * rho * rho + 0.5;
    for (int chir : {1, -1}) {
      DBuf pc(sizeof(double) * 4, s);
      if (!pc.p) return fail(LQ_ENOMEM, "eigensolver");
      const double q[4] = {top - 2.0 * rho * rho, -rho * rho, (double)chir, 1.0};  // top - H_s
      hipMemcpyAsync(pc.p, q, sizeof(q), hipMemcpyHostToDevice, s);
      Vec t = make_vec(g, 64, 12, 1, 2, 0, s);
      if (!t.ok()) return fail(LQ_ENOMEM, "eigensolver");
      Blas bl;
      if ((e = blas_prepare(c, bl, g, 2, nev, s))) return e;
      // the sign function in FP64, or in FP32 for a loose target (tol >= 1e-6:
      // enough for a deflation guess, at a third of the cost)
      const int ep = tol >= 1e-6 ? 32 : 64;
      Vec t32i = make_vec(g, ep, 12, 1, 2, 0, s), t32o = make_vec(g, ep, 12, 1, 2, 0, s);
      if (!t32i.ok() || !t32o.ok()) return fail(LQ_ENOMEM, "eigensolver");
      auto sign_at = [&](Vec& out64, const Vec& in64) -> int {
        if (ep == 64) return sign_apply(env, 64, out64, in64);
        int r = vec_copy(t32i, in64);
        if (!r) r = sign_apply(env, ep, t32o, t32i);
        return r ? r : vec_copy(out64, t32o);
      };
      OpFn A = [&](Vec& out, const Vec& in) {
        int r = sign_at(t, in);
        return r ? r : bl.plc(const_cast<Vec*>(&in), &t, &out, pc.as<double>());
      };
      IrlOut io;
      const int r = irl(c, g, s, A, [&](Vec& v) { return random_start(g, s, v, chir > 0 ? 778 : 779, chir); }, nev,
                        k, m, tol, max_restarts, V, io);
      if (r && r != LQ_ENOCONV) return r;
      apps += io.applications;
      restarts += io.restarts;
      // H_s eigenpairs: Rayleigh-Ritz with H_s (same vectors, eigenvalues top - theta)
      DBuf ph(sizeof(double) * 4, s);
      const double qh[4] = {2.0 * rho * rho, rho * rho, (double)chir, 1.0};
      hipMemcpyAsync(ph.p, qh, sizeof(qh), hipMemcpyHostToDevice, s);
      Vec tt = make_vec(g, 64, 12, nev, 2, 0, s);
      DBuf phn(sizeof(double) * 4 * nev, s);
      if (!ph.p || !tt.ok() || !phn.p) return fail(LQ_ENOMEM, "eigensolver");
      std::vector<double> qn((size_t)4 * nev);
      for (int l = 0; l < nev; ++l) std::memcpy(&qn[(size_t)4 * l], qh, sizeof(qh));
      hipMemcpyAsync(phn.p, qn.data(), sizeof(double) * qn.size(), hipMemcpyHostToDevice, s);
      Vec ti = make_vec(g, ep, 12, nev, 2, 0, s), to = make_vec(g, ep, 12, nev, 2, 0, s);
      if (!ti.ok() || !to.ok()) return fail(LQ_ENOMEM, "eigensolver");
      OpFn Hs = [&](Vec& out, const Vec& in) {
        Vec tv = view(tt, 0, in.ncol);
        int r2 = 0;
        if (ep == 64) {
          r2 = sign_apply(env, 64, tv, in);
        } else {
          Vec tiv = view(ti, 0, in.ncol), tov = view(to, 0, in.ncol);
          r2 = vec_copy(tiv, in);
          if (!r2) r2 = sign_apply(env, ep, tov, tiv);
          if (!r2) r2 = vec_copy(tv, tov);
        }
        return r2 ? r2 : bl.plc(const_cast<Vec*>(&in), &tv, &out, phn.as<double>());
      };
      std::vector<double> mu, res;
      if ((e = rayleigh_ritz(env, V, nev, mu, res, Hs))) return e;
      EigSet es;
      es.which = LQ_EIG_OVERLAP;
      es.rho = rho;
      es.chir = chir;
      es.vals = mu;
      es.res = res;
      const size_t bytes = vec_bytes(g, 64, 12, nev, 2);
      if (hipMalloc(&es.vecs, bytes) != hipSuccess) return fail(LQ_ENOMEM, "eigenvector storage");
      if (hipMemcpyAsync(es.vecs, V.f.data, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(LQ_EDEVICE, "copy");
      es.n = nev;
      sets.push_back(std::move(es));
      all_vals.insert(all_vals.end(), mu.begin(), mu.end());
      all_res.insert(all_res.end(), res.begin(), res.end());
      for (double rr : res)
        if (!(rr <= tol * 4.0 * rho * rho)) status = LQ_ENOCONV;
    }
  } else {
    return fail(LQ_EINVAL, "unknown eigenproblem");
  }
  if (which == LQ_EIG_HW) {
    const size_t bytes = vec_bytes(g, 64, 12, nev, 2);
    if (hipMalloc(&sets[0].vecs, bytes) != hipSuccess) return fail(LQ_ENOMEM, "eigenvector storage");
    if (hipMemcpyAsync(sets[0].vecs, V.f.data, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(LQ_EDEVICE, "copy");
    sets[0].n = nev;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "eigensolver");
  {
    std::lock_guard<std::mutex> lk(f->mtx);
    for (auto& es : sets) {
      auto key = std::make_tuple(es.which, es.rho, es.chir);
      auto it = f->eig.find(key);
      if (it != f->eig.end() && it->second.vecs) hipFree(it->second.vecs);
      f->eig[key] = std::move(es);
    }
  }
  if (evals) std::memcpy(evals, all_vals.data(), sizeof(double) * all_vals.size());
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = restarts;
    st->n_apply = apps;
    st->true_rel_res = all_res.empty() ? 0 : *std::max_element(all_res.begin(), all_res.end());
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st->status = status;
  }
  if (status == LQ_ENOCONV) return fail(LQ_ENOCONV, "eigensolver: residuals above the tolerance");
  return LQ_OK;
}

const EigSet* find_eigs(lq_field* f, int which, double rho, int chir) {
  std::lock_guard<std::mutex> lk(f->mtx);
  auto it = f->eig.find(std::make_tuple(which, rho, chir));
  return it == f->eig.end() ? nullptr : &it->second;
}

// ------------------------------------------------------------------ use of the low modes
// out = P ... with P = 1 - U U^H over the first n columns of U (FP64 columns
// of v in place); coef (device, n x ncol complex) receives U^H v if given
int project_out(lq_ctx* c, const Geom& g, hipStream_t s, const EigSet& es, int n, Vec& v, void* coef) {
  rocblas_handle h = rb_handle(c, s);
  if (!h) return fail(LQ_EDEVICE, "rocBLAS handle");
  const int64_t N = col_len(g);
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0}, mone = {-1.0, 0.0};
  const rocblas_double_complex* U = (const rocblas_double_complex*)es.vecs;
  // U^H v column by column (a matrix-vector product per column: the library's
  // gemm is slow for this shape, two tiny dimensions and one of ~1e7)
  for (int col = 0; col < v.ncol; ++col)
    if (rocblas_zgemv(h, rocblas_operation_conjugate_transpose, N, n, &one, U, N, colp(v, col), 1, &zero,
                      (rocblas_double_complex*)coef + (size_t)col * n, 1) != rocblas_status_success)
      return fail(LQ_EDEVICE, "rocBLAS gemv");
  if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, N, v.ncol, n, &mone, U, N,
                    (const rocblas_double_complex*)coef, n, &one, colp(v, 0), N) != rocblas_status_success)
    return fail(LQ_EDEVICE, "rocBLAS gemm");
  return 0;
}

// v += U diag(f) coef: adds back the low-mode part with weights f_i (host array)
int add_modes(lq_ctx* c, const Geom& g, hipStream_t s, const EigSet& es, int n, const std::vector<double>& wts,
              Vec& v, void* coef) {
  rocblas_handle h = rb_handle(c, s);
  if (!h) return fail(LQ_EDEVICE, "rocBLAS handle");
  const int64_t N = col_len(g);
  std::vector<zc> cf((size_t)n * v.ncol);
  hipMemcpyAsync(cf.data(), coef, sizeof(zc) * cf.size(), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "coefficients");
  for (int col = 0; col < v.ncol; ++col)
    for (int i = 0; i < n; ++i) cf[(size_t)col * n + i] *= wts[(size_t)col * n + i];
  hipMemcpyAsync(coef, cf.data(), sizeof(zc) * cf.size(), hipMemcpyHostToDevice, s);
  const rocblas_double_complex one = {1.0, 0.0};
  if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, N, v.ncol, n, &one,
                    (const rocblas_double_complex*)es.vecs, N, (const rocblas_double_complex*)coef, n, &one,
                    colp(v, 0), N) != rocblas_status_success)
    return fail(LQ_EDEVICE, "rocBLAS gemm");
  return 0;
}

}  // namespace lq
