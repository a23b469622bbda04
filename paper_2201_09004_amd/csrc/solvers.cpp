// Krylov drivers (host control, device data and scalars):
//   * mixed-precision CG with reliable updates (Wilson normal equations,
//     HISQ per-shift refinement, overlap outer solve);
//   * mixed-precision BiCGStab with reliable updates on the even-odd Schur
//     system of the twisted-clover operator (sec. 2.1, Table 2);
//   * multi-shift CG for several staggered masses at once (sec. 2.3 cites
//     the shifted Krylov solvers; Table 3 uses CG for HISQ);
//   * FP64 Lanczos for the spectral interval of H_W^2 (sec. 2.3).
// Every solution is accepted only when its FP64 true residual, computed with
// the FP64 operator of the full (unpreconditioned) system, meets the target.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>

#include "lq_internal.h"
#include "solver_util.h"

// precision of the HISQ multi-shift stage when the sloppy precision is FP16,
// and its target relative residual in FP32
#ifndef LQ_MS_PREC16
#define LQ_MS_PREC16 32
#endif
#ifndef LQ_MS_TOL32
#define LQ_MS_TOL32 1e-8
#endif

namespace lq {


// LQ_VERBOSE=1: the solvers report each reliable update and each overlap
// correction pass on stderr (progress of long solves)
static bool verbose() {
  static const bool v = [] {
    const char* e = getenv("LQ_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

// timing records of the multi-shift vector kernels with their algorithmic
// bytes: ms_xr reads r and A p and writes r (base columns); ms_p reads r once
// and, per shift column, reads p and x and writes both
struct MsProf {
  Prof all, one;
  char name[32];
  static double bytes(const MsArgs& M, bool p) {
    const double sb = (double)site_bytes(M.prec, M.nc) + (sep_norm(M.prec, M.nc) ? 4 : 0);
    const double cols = p ? M.nrhs + 4.0 * M.nshift * M.nrhs : 3.0 * M.nrhs;
    return cols * M.npar * M.Vh * sb;
  }
  MsProf(lq_ctx* c, const MsArgs& M, bool p, hipStream_t s)
      : all(c, "blas", s, bytes(M, p)),
        one(c, (snprintf(name, sizeof(name), "ms%d_%s", M.prec, p ? "p" : "xr"), name), s, bytes(M, p)) {}
};

namespace {
struct Counters {
  int iters = 0, reliable = 0, restarts = 0;
  int fault = 0;
};
}  // namespace

int col_norms(Blas& bl, Vec& v, std::vector<double>& out) {
  State st(v.ncol, bl.s);
  if (!st.ok()) return fail(LQ_ENOMEM, "state");
  int r = bl.op(OP_NORM2, &v);
  if (r) return r;
  if (launch_scalar(SC_SET_RR, bl.partial, bl.gridx, v.ncol, st.d(), bl.s)) return fail(LQ_EDEVICE, "scalar");
  if ((r = st.pull())) return r;
  out.resize(v.ncol);
  for (int c = 0; c < v.ncol; ++c) out[c] = st.h(c, ST_RR);
  return 0;
}

int rel_residual(Blas& bl, const OpFn& A, Vec& x, Vec& b, std::vector<double>& res, const Geom& g) {
  Vec q = make_vec(g, 64, b.nc, b.ncol, b.npar, b.par0, bl.s);
  if (!q.ok()) return fail(LQ_ENOMEM, "residual buffer");
  int r = A(q, x);
  if (r) return r;
  if ((r = bl.op(OP_XMY_NORM, &b, &q))) return r;
  State st(b.ncol, bl.s);
  if (launch_scalar(SC_SET_RR, bl.partial, bl.gridx, b.ncol, st.d(), bl.s)) return fail(LQ_EDEVICE, "scalar");
  if ((r = st.pull())) return r;
  std::vector<double> bb;
  if ((r = col_norms(bl, b, bb))) return r;
  res.resize(b.ncol);
  for (int c = 0; c < b.ncol; ++c) res[c] = bb[c] > 0 ? std::sqrt(st.h(c, ST_RR) / bb[c]) : 0.0;
  return 0;
}

namespace {

// Per-column parameters of the operator (e.g. one mass per column) that have
// to follow the columns when the solver reorders them.
struct ColParam {
  std::vector<double> host;  // [ncol][stride]
  double* dev = nullptr;
  hipStream_t s = nullptr;
  int stride = 1;
  void swap(int a, int c) {
    for (int k = 0; k < stride; ++k) std::swap(host[(size_t)a * stride + k], host[(size_t)c * stride + k]);
  }
  int upload() const {
    return hipMemcpyAsync(dev, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, s) == hipSuccess
               ? 0
               : fail(LQ_EDEVICE, "column parameters");
  }
};

// Keeps the active columns of a batched solver in slots [0, na): a converged
// column is exchanged with the last active one in every listed vector, in the
// solver state and in the per-column host arrays and operator parameters.
// The exchanges applied to the caller's x and b are undone by restore().
struct Compactor {
  State& st;
  Vec& x;
  Vec& b;
  std::vector<Vec*> vecs;                    // solver-owned vectors that carry column data
  std::vector<std::vector<double>*> arrays;  // per-column host values
  ColParam* cp = nullptr;
  int na = 0;
  std::vector<std::pair<int, int>> swaps;

  int swap(int a, int c) {
    if (a == c) return 0;
    int e = 0;
    if ((e = vec_swap_cols(x, a, c)) || (e = vec_swap_cols(b, a, c))) return e;
    for (Vec* v : vecs)
      if ((e = vec_swap_cols(*v, a, c))) return e;
    for (int k = 0; k < ST_STRIDE; ++k) std::swap(st.h(a, k), st.h(c, k));
    for (auto* arr : arrays) std::swap((*arr)[a], (*arr)[c]);
    if (cp) cp->swap(a, c);
    swaps.emplace_back(a, c);
    return 0;
  }
  // moves columns whose ST_ACTIVE is 0 behind the active ones (the host state
  // must be current for [0, na)); pushes the state and the parameters
  int compact() {
    int e = 0;
    for (int c = na - 1; c >= 0; --c) {
      if (st.h(c, ST_ACTIVE) != 0.0) continue;
      if ((e = swap(c, na - 1))) return e;
      --na;
    }
    if ((e = st.push())) return e;
    if (cp && (e = cp->upload())) return e;
    return 0;
  }
  int restore() {
    int e = 0;
    for (auto it = swaps.rbegin(); it != swaps.rend(); ++it) {
      if ((e = vec_swap_cols(x, it->first, it->second)) || (e = vec_swap_cols(b, it->first, it->second))) return e;
      if (cp) cp->swap(it->first, it->second);
    }
    if (cp && !swaps.empty() && (e = cp->upload())) return e;
    swaps.clear();
    return 0;
  }
};

// A sloppy operator that also returns reductions as partials over 64-site
// tiles ([col][tile][4]): mode 1 <in, out> (CG), mode 2 <out, in> and |out|^2 (BiCGStab)
using FusedFn = std::function<int(Vec& out, const Vec& in, int mode, double* red)>;

// Mixed-precision CG with reliable updates on a Hermitian positive-definite A.
// x, b: FP64.  Columns stop when the FP64 residual of A meets tol[c] |b_c|.
// Converged columns are moved behind the active ones (columns of every
// vector, the solver state and `cp` are exchanged together), so the operator
// and the vector kernels only run over the columns still iterating; x and b
// are put back in their original order before returning.  A_hi and A_lo
// receive views of the active columns.
int cg_mixed(Blas& bl, const Geom& g, const OpFn& A_hi, const OpFn& A_lo, int plo, Vec& x, Vec& b,
             const std::vector<double>& tol_in, int maxiter, double delta, Counters& cnt, ColParam* cp = nullptr,
             const FusedFn* A_fused = nullptr) {
  const int n = b.ncol, nc = b.nc, npar = b.npar, par0 = b.par0;
  hipStream_t s = bl.s;
  // A_fused: the sloppy operator with <p, A p> from its stencil epilogue
  const int fused_tiles = (npar * g.Vh + 63) / 64;
  DBuf redbuf(A_fused ? sizeof(double) * 4 * (size_t)fused_tiles * n : 0, s);
  if (A_fused && !redbuf.p) return fail(LQ_ENOMEM, "reduction partials");
  Vec r = make_vec(g, 64, nc, n, npar, par0, s);
  Vec q64 = make_vec(g, 64, nc, n, npar, par0, s);
  Vec rs = make_vec(g, plo, nc, n, npar, par0, s);
  Vec p = make_vec(g, plo, nc, n, npar, par0, s);
  Vec q = make_vec(g, plo, nc, n, npar, par0, s);
  Vec xs = make_vec(g, plo, nc, n, npar, par0, s);
  State st(n, s);
  if (!r.ok() || !q64.ok() || !rs.ok() || !p.ok() || !q.ok() || !xs.ok() || !st.ok())
    return fail(LQ_ENOMEM, "cg buffers");
  std::vector<double> bb, tol(tol_in);
  int e = col_norms(bl, b, bb);
  if (e) return e;
  int na = n;  // active columns occupy slots [0, na)
  // r = b - A x (FP64) on the active columns
  auto true_res = [&]() -> int {
    Vec qv = view(q64, 0, na), xv = view(x, 0, na), bv = view(b, 0, na);
    int rr = A_hi(qv, xv);
    if (rr) return rr;
    if ((rr = bl.op(OP_XMY_NORM, &bv, &qv))) return rr;
    std::swap(r, q64);
    if (launch_scalar(SC_SET_RR, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    return 0;
  };
  std::vector<double> maxrr(n), rr_chk(n);  // rr_chk: |r|^2 at the last host check
  Compactor cm{st, x, b, {&r, &rs, &p, &xs}, {&bb, &tol, &maxrr, &rr_chk}, cp, n, {}};
  auto compact = [&]() -> int {
    const int e2 = cm.compact();
    na = cm.na;
    return e2;
  };
  for (int c = 0; c < n; ++c) {
    for (int k = 0; k < ST_STRIDE; ++k) st.h(c, k) = 0.0;
    st.h(c, ST_ACTIVE) = 1.0;
  }
  if ((e = st.push())) return e;
  if ((e = true_res())) return e;
  if ((e = vec_copy(rs, r)) || (e = vec_copy(p, r)) || (e = vec_zero(xs))) return e ? e : fail(LQ_EDEVICE, "copy");
  if ((e = st.pull())) return e;
  for (int c = 0; c < n; ++c) {
    maxrr[c] = rr_chk[c] = st.h(c, ST_RR);
    const bool act = st.h(c, ST_RR) > tol[c] * tol[c] * bb[c] && bb[c] > 0;
    st.h(c, ST_ACTIVE) = act ? 1.0 : 0.0;
  }
  if ((e = compact())) return e;
  bool dirty = false;  // xs holds un-folded updates
  // Host checks of the residual norms may be deferred while every column is
  // predicted to be far from its next update-rule threshold (positivity
  // restarts happen on the device, so FP16 sloppy vectors defer as well).
  const bool defer = cnt.fault == 0;
  int skip = 0, since = 0;
  int it = 0;
  for (; it < maxiter && na > 0; ++it) {
    Vec pv = view(p, 0, na), qv = view(q, 0, na), xsv = view(xs, 0, na), rsv = view(rs, 0, na);
    if (A_fused) {
      if ((e = (*A_fused)(qv, pv, 1, redbuf.as<double>()))) return e;
      if (launch_scalar(SC_CG_ALPHA, redbuf.as<double>(), fused_tiles, na, st.d(), s))
        return fail(LQ_EDEVICE, "scalar");
    } else {
      if ((e = A_lo(qv, pv))) return e;
      if ((e = bl.op(OP_DOT, &pv, &qv))) return e;
      if (launch_scalar(SC_CG_ALPHA, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    }
    if ((e = bl.op(OP_CG, &pv, &qv, &xsv, &rsv, nullptr, st.d(), ST_ALPHA, ST_ALPHA))) return e;
    if (launch_scalar(SC_CG_BETA, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    ++since;
    if (defer && skip > 0 && it < maxiter - 1) {
      --skip;
      dirty = true;
      if ((e = bl.op(OP_XPAY, &rsv, &pv, nullptr, nullptr, nullptr, st.d(), ST_BETA, ST_BETA))) return e;
      continue;
    }
    if (cnt.fault == 1 && it == 0) {
      // injected NaN in the first reduction (host-forced test of the numeric guard)
      if ((e = st.pull(na))) return e;
      st.h(0, ST_FLAG) = 2.0;
      if ((e = st.push(na))) return e;
    }
    dirty = true;
    if ((e = st.pull(na))) return e;
    UpdateRule rule;
    double nrst = 0.0;  // direction restarts (taken on the device by SC_CG_BETA)
    for (int c = 0; c < na; ++c) {
      if (st.h(c, ST_FLAG) == 2.0) return fail(LQ_ENUMERIC, "NaN/Inf in a CG reduction");
      nrst += st.h(c, ST_NRST);
      const double rr = st.h(c, ST_RR);
      maxrr[c] = std::max(maxrr[c], rr);
      rule.column(rr, maxrr[c], tol[c] * tol[c] * bb[c], delta);
    }
    for (int c = na; c < n; ++c) nrst += st.h(c, ST_NRST);
    if (nrst > 50.0 * n) return fail(LQ_EBREAKDOWN, "CG keeps losing positivity of <p, A p>");
    const bool update = rule.fire();
    if (defer && !update) {
      double k = 8.0;
      for (int c = 0; c < na; ++c)
        k = std::min(k, 0.5 * iters_to_event(st.h(c, ST_RR), rr_chk[c], since, maxrr[c], tol[c] * tol[c] * bb[c],
                                             delta));
      skip = (int)k;
    }
    for (int c = 0; c < na; ++c) rr_chk[c] = st.h(c, ST_RR);
    since = 0;
    if (update && rule.converged_few() && it < maxiter - 1) {
      // Only a few columns are below their targets: fold every column's sloppy
      // updates into x, move those columns to slots [0, m) and recompute the
      // FP64 residual of these alone; the others keep iterating untouched.
      ++cnt.reliable;
      if ((e = launch_axpy_mixed(x.f, 64, xs.f, plo, nc, na, npar, g.Vh, s))) return fail(LQ_EDEVICE, "axpy");
      if ((e = vec_zero(xsv))) return e;
      dirty = false;
      int m = 0;
      for (int c = 0; c < na; ++c)
        if (st.h(c, ST_RR) < tol[c] * tol[c] * bb[c]) {
          if ((e = cm.swap(c, m))) return e;
          ++m;
        }
      if ((e = st.push(na))) return e;
      if (cp && (e = cp->upload())) return e;
      {
        Vec qv = view(q64, 0, m), xv = view(x, 0, m), bv = view(b, 0, m), rv = view(r, 0, m), rsm = view(rs, 0, m);
        if ((e = A_hi(qv, xv)) || (e = bl.op(OP_XMY_NORM, &bv, &qv)) || (e = vec_copy(rv, qv))) return e;
        if (launch_scalar(SC_SET_RR, bl.partial, bl.gridx, m, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
        if ((e = vec_copy(rsm, rv))) return e;
      }
      if ((e = st.pull(na))) return e;
      for (int c = 0; c < m; ++c) {
        const double rr = st.h(c, ST_RR);
        if (!std::isfinite(rr)) return fail(LQ_ENUMERIC, "NaN/Inf in the true residual");
        maxrr[c] = rr_chk[c] = rr;
        if (rr <= tol[c] * tol[c] * bb[c]) {
          st.h(c, ST_ACTIVE) = 0.0;
          st.h(c, ST_BETA) = 0.0;
        }
      }
      if ((e = compact())) return e;
    } else if (update || it == maxiter - 1) {
      ++cnt.reliable;
      if ((e = launch_axpy_mixed(x.f, 64, xs.f, plo, nc, na, npar, g.Vh, s))) return fail(LQ_EDEVICE, "axpy");
      if ((e = vec_zero(xsv))) return e;
      dirty = false;
      // keep the CG direction scalars (beta) computed in sloppy precision
      if ((e = true_res())) return e;
      {
        Vec rv = view(r, 0, na);
        if ((e = vec_copy(rsv, rv))) return e;
      }
      if ((e = st.pull(na))) return e;
      for (int c = 0; c < na; ++c) {
        const double rr = st.h(c, ST_RR);
        if (!std::isfinite(rr)) return fail(LQ_ENUMERIC, "NaN/Inf in the true residual");
        maxrr[c] = rr_chk[c] = rr;
        if (rr <= tol[c] * tol[c] * bb[c]) {
          st.h(c, ST_ACTIVE) = 0.0;
          st.h(c, ST_BETA) = 0.0;
        }
      }
      if (verbose()) {
        double wr = 0.0;
        for (int c = 0; c < na; ++c) wr = std::max(wr, bb[c] > 0 ? std::sqrt(st.h(c, ST_RR) / bb[c]) : 0.0);
        fprintf(stderr, "[lq] cg iter %d: reliable update %d, %d active columns, worst rel. residual %.3e\n",
                cnt.iters + it + 1, cnt.reliable, na, wr);
      }
      if ((e = compact())) return e;
    }
    if (na == 0) {
      ++it;
      break;
    }
    Vec rsn = view(rs, 0, na), pn = view(p, 0, na);
    if ((e = bl.op(OP_XPAY, &rsn, &pn, nullptr, nullptr, nullptr, st.d(), ST_BETA, ST_BETA))) return e;
  }
  if (dirty && na > 0) {
    if ((e = launch_axpy_mixed(x.f, 64, xs.f, plo, nc, na, npar, g.Vh, s))) return fail(LQ_EDEVICE, "axpy");
  }
  const int left = na;
  // original column order of x and b (and of the caller's column parameters)
  if ((e = cm.restore())) return e;
  cnt.iters += it;
  return left > 0 ? LQ_ENOCONV : LQ_OK;
}

// Mixed-precision BiCGStab with reliable updates for a non-Hermitian M.
// M_fused (optional): the sloppy operator with the fused reductions <out, in>
// and |out|^2 (mode 2) as partials over 64-site tiles.

int bicgstab_mixed(Blas& bl, const Geom& g, const OpFn& M_hi, const OpFn& M_lo, int plo, Vec& x, Vec& b,
                   const std::vector<double>& tol_in, int maxiter, double delta, Counters& cnt,
                   const FusedFn* M_fused = nullptr) {
  const int n = b.ncol, nc = b.nc, npar = b.npar, par0 = b.par0;
  hipStream_t s = bl.s;
  const int fused_tiles = (npar * g.Vh + 63) / 64;
  DBuf redbuf(M_fused ? sizeof(double) * 4 * (size_t)fused_tiles * n : 0, s);
  if (M_fused && !redbuf.p) return fail(LQ_ENOMEM, "reduction partials");
  Vec r = make_vec(g, 64, nc, n, npar, par0, s);
  Vec q64 = make_vec(g, 64, nc, n, npar, par0, s);
  Vec rs = make_vec(g, plo, nc, n, npar, par0, s);
  Vec rhat = make_vec(g, plo, nc, n, npar, par0, s);
  Vec p = make_vec(g, plo, nc, n, npar, par0, s);
  Vec v = make_vec(g, plo, nc, n, npar, par0, s);
  Vec t = make_vec(g, plo, nc, n, npar, par0, s);
  Vec xs = make_vec(g, plo, nc, n, npar, par0, s);
  State st(n, s);
  if (!r.ok() || !q64.ok() || !rs.ok() || !rhat.ok() || !p.ok() || !v.ok() || !t.ok() || !xs.ok() || !st.ok())
    return fail(LQ_ENOMEM, "bicgstab buffers");
  std::vector<double> bb, tol(tol_in);
  int e = col_norms(bl, b, bb);
  if (e) return e;
  std::vector<double> maxrr(n), rr_chk(n);  // rr_chk: |r|^2 at the last host check
  // active columns occupy slots [0, cm.na); v carries column data from one
  // iteration's M p into the same iteration's p update, across a compaction
  Compactor cm{st, x, b, {&rs, &rhat, &p, &v, &xs}, {&bb, &tol, &maxrr, &rr_chk}, nullptr, n, {}};
  auto V = [&](Vec& f) { return view(f, 0, cm.na); };
  auto true_res = [&]() -> int {
    Vec qv = V(q64), xv = V(x), bv = V(b);
    int rr = M_hi(qv, xv);
    if (rr) return rr;
    if ((rr = bl.op(OP_XMY_NORM, &bv, &qv))) return rr;
    std::swap(r, q64);
    return 0;
  };
  // (re)start: r = b - M x, rhat = r, p = r, rho = <rhat, r>
  auto restart = [&]() -> int {
    int rr = true_res();
    if (rr) return rr;
    Vec rv = V(r), rsv = V(rs), rhv = V(rhat), pv = V(p);
    if ((rr = vec_copy(rsv, rv)) || (rr = vec_copy(rhv, rv)) || (rr = vec_copy(pv, rv))) return rr;
    if ((rr = bl.op(OP_DOT_NORM, &rsv, &rhv))) return rr;
    if (launch_scalar(SC_SET_RHO_RR, bl.partial, bl.gridx, cm.na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    return 0;
  };
  for (int c = 0; c < n; ++c) {
    for (int k = 0; k < ST_STRIDE; ++k) st.h(c, k) = 0.0;
    st.h(c, ST_ACTIVE) = 1.0;
  }
  if ((e = st.push())) return e;
  if ((e = vec_zero(xs))) return e;
  if ((e = restart())) return e;
  if ((e = st.pull())) return e;
  for (int c = 0; c < n; ++c) {
    maxrr[c] = rr_chk[c] = st.h(c, ST_RR);
    const bool act = st.h(c, ST_RR) > tol[c] * tol[c] * bb[c] && bb[c] > 0;
    st.h(c, ST_ACTIVE) = act ? 1.0 : 0.0;
  }
  if ((e = cm.compact())) return e;
  bool dirty = false;
  // Host reads of the state may be deferred, as in CG, while every column is
  // predicted to be far from its next update-rule threshold.  A breakdown in a
  // skipped iteration leaves its column frozen (zero steps, sticky flag) until
  // the next read restarts it.
  const bool defer = cnt.fault == 0;
  int skip = 0, since = 0;
  int it = 0;
  for (; it < maxiter && cm.na > 0; ++it) {
    const int na = cm.na;
    Vec pv = V(p), vv = V(v), tv = V(t), rsv = V(rs), rhv = V(rhat), xsv = V(xs);
    // <rhat, v> by a separate pass: fused into the stencil it measured slower
    // than the pass, since the extra rhat stream raises the register pressure
    // of the already heaviest epilogue
    if ((e = M_lo(vv, pv))) return e;
    if ((e = bl.op(OP_DOT, &rhv, &vv))) return e;
    if (launch_scalar(SC_BICG_ALPHA, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if ((e = bl.op(OP_AXMY, &vv, &rsv, nullptr, nullptr, nullptr, st.d(), ST_ALPHA, ST_ALPHA))) return e;
    if (M_fused) {
      // <t, s> and |t|^2 computed by the stencil that produces t = M s
      if ((e = (*M_fused)(tv, rsv, 2, redbuf.as<double>()))) return e;
      if (launch_scalar(SC_BICG_OMEGA, redbuf.as<double>(), fused_tiles, na, st.d(), s))
        return fail(LQ_EDEVICE, "scalar");
    } else {
      if ((e = M_lo(tv, rsv))) return e;
      if ((e = bl.op(OP_DOT_NORM, &tv, &rsv))) return e;
      if (launch_scalar(SC_BICG_OMEGA, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    }
    if ((e = bl.op(OP_BICG_XR, &pv, &rsv, &tv, &xsv, &rhv, st.d(), ST_ALPHA, ST_OMEGA))) return e;
    if (launch_scalar(SC_BICG_BETA, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    dirty = true;
    ++since;
    if (defer && skip > 0 && it < maxiter - 1) {
      --skip;
      if ((e = bl.op(OP_BICG_P, &rsv, &vv, &pv, nullptr, nullptr, st.d(), ST_BETA, ST_OMEGA))) return e;
      continue;
    }
    if ((e = st.pull(na))) return e;
    bool breakdown = false;
    UpdateRule rule;
    for (int c = 0; c < na; ++c) {
      if (st.h(c, ST_FLAG) == 2.0) return fail(LQ_ENUMERIC, "NaN/Inf in a BiCGStab reduction");
      if (st.h(c, ST_FLAG) == 1.0) breakdown = true;
      const double rr = st.h(c, ST_RR);
      if (!std::isfinite(rr)) return fail(LQ_ENUMERIC, "NaN/Inf residual");
      maxrr[c] = std::max(maxrr[c], rr);
      rule.column(rr, maxrr[c], tol[c] * tol[c] * bb[c], delta);
    }
    const bool update = rule.fire();
    if (defer && !update && !breakdown) {
      double k = 8.0;
      for (int c = 0; c < na; ++c)
        k = std::min(k, 0.5 * iters_to_event(st.h(c, ST_RR), rr_chk[c], since, maxrr[c], tol[c] * tol[c] * bb[c],
                                             delta));
      skip = (int)k;
    }
    for (int c = 0; c < na; ++c) rr_chk[c] = st.h(c, ST_RR);
    since = 0;
    if (update || breakdown || it == maxiter - 1) {
      ++cnt.reliable;
      if ((e = launch_axpy_mixed(x.f, 64, xs.f, plo, nc, na, npar, g.Vh, s))) return fail(LQ_EDEVICE, "axpy");
      if ((e = vec_zero(xsv))) return e;
      dirty = false;
      if (breakdown) {
        ++cnt.restarts;
        if (cnt.restarts > 20) return fail(LQ_EBREAKDOWN, "BiCGStab breakdown persists after restarts");
        for (int c = 0; c < na; ++c) st.h(c, ST_FLAG) = 0.0;
        if ((e = st.push(na))) return e;
        if ((e = restart())) return e;
      } else {
        if ((e = true_res())) return e;
        Vec rv = V(r);
        if ((e = vec_copy(rsv, rv))) return e;
        if ((e = bl.op(OP_DOT_NORM, &rsv, &rhv))) return e;
        if (launch_scalar(SC_SET_RHO_RR, bl.partial, bl.gridx, na, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
      }
      if ((e = st.pull(na))) return e;
      for (int c = 0; c < na; ++c) {
        const double rr = st.h(c, ST_RR);
        maxrr[c] = rr_chk[c] = rr;
        if (rr <= tol[c] * tol[c] * bb[c]) st.h(c, ST_ACTIVE) = 0.0;
      }
      if ((e = cm.compact())) return e;
      if (breakdown) continue;  // p = r already
    }
    if (cm.na == 0) {
      ++it;
      break;
    }
    Vec rsn = V(rs), vn = V(v), pn = V(p);
    if ((e = bl.op(OP_BICG_P, &rsn, &vn, &pn, nullptr, nullptr, st.d(), ST_BETA, ST_OMEGA))) return e;
  }
  if (dirty && cm.na > 0) {
    if ((e = launch_axpy_mixed(x.f, 64, xs.f, plo, nc, cm.na, npar, g.Vh, s))) return fail(LQ_EDEVICE, "axpy");
  }
  const int left = cm.na;
  if ((e = cm.restore())) return e;
  cnt.iters += it;
  return left > 0 ? LQ_ENOCONV : LQ_OK;
}

// Flexible GCR (generalised conjugate residual, restarted after kmax
// directions) in FP64 on a non-Hermitian M with a variable preconditioner:
// every outer direction z_k = K(r) may come from a different preconditioner
// (a short sloppy Krylov solve, a multigrid cycle), so M z_k is orthogonalised
// against the earlier M z_j (modified Gram-Schmidt, applied to z_k alike) and
// the residual is minimised over the span.  The outer recurrence is FP64, so r
// stays the true residual up to rounding; it is recomputed at every restart.
// K may add to cnt; the outer steps are returned in *steps.
using PrecFn = std::function<int(Vec& z, Vec& r, Counters& cnt)>;

int fgcr(Blas& bl, const Geom& g, const OpFn& M_hi, const PrecFn& K, Vec& x, Vec& b,
         const std::vector<double>& tol_in, int maxiter, Counters& cnt, int kmax, const char* tag,
         int* steps = nullptr) {
  const int n = b.ncol, nc = b.nc, npar = b.npar, par0 = b.par0;
  hipStream_t s = bl.s;
  Vec r = make_vec(g, 64, nc, n, npar, par0, s), q = make_vec(g, 64, nc, n, npar, par0, s);
  std::vector<Vec> Z, W;
  for (int k = 0; k < kmax; ++k) {
    Z.push_back(make_vec(g, 64, nc, n, npar, par0, s));
    W.push_back(make_vec(g, 64, nc, n, npar, par0, s));
    if (!Z.back().ok() || !W.back().ok()) return fail(LQ_ENOMEM, "gcr buffers");
  }
  State st(n, s);
  if (!r.ok() || !q.ok() || !st.ok()) return fail(LQ_ENOMEM, "gcr buffers");
  for (int c = 0; c < n; ++c) {
    for (int k = 0; k < ST_STRIDE; ++k) st.h(c, k) = 0.0;
    st.h(c, ST_ACTIVE) = 1.0;
  }
  int e = st.push();
  if (e) return e;
  std::vector<double> bb, tol(tol_in), rr;
  if ((e = col_norms(bl, b, bb))) return e;
  auto true_res = [&]() -> int {
    int rs = M_hi(q, x);
    if (rs) return rs;
    if ((rs = bl.op(OP_XMY_NORM, &b, &q))) return rs;
    std::swap(r, q);
    return 0;
  };
  auto converged = [&]() -> bool {
    for (int c = 0; c < n; ++c)
      if (bb[c] > 0 && rr[c] > tol[c] * tol[c] * bb[c]) return false;
    return true;
  };
  // a per-column coefficient in the state (ST_AUX) from the partials of a reduction
  auto to_aux = [&]() -> int {
    return launch_scalar(SC_DOT_TO_AUX, bl.partial, bl.gridx, n, st.d(), s) ? fail(LQ_EDEVICE, "scalar") : 0;
  };
  if ((e = true_res()) || (e = col_norms(bl, r, rr))) return e;
  int it = 0, k = 0;
  while (it < maxiter && !converged()) {
    if (k == kmax) {  // restart from the true residual
      ++cnt.reliable;
      if ((e = true_res()) || (e = col_norms(bl, r, rr))) return e;
      k = 0;
      if (converged()) break;
    }
    // z_k = K(r)
    Vec& zk = Z[k];
    Vec& wk = W[k];
    if ((e = K(zk, r, cnt))) return e;
    // w_k = M z_k, orthogonal to the earlier w_j (same combination on z_k)
    if ((e = M_hi(wk, zk))) return e;
    for (int j = 0; j < k; ++j) {
      if ((e = bl.op(OP_DOT, &W[j], &wk)) || (e = to_aux())) return e;
      if ((e = bl.op(OP_AXMY, &W[j], &wk, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
          (e = bl.op(OP_AXMY, &Z[j], &zk, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)))
        return e;
    }
    std::vector<double> ww;
    if ((e = col_norms(bl, wk, ww))) return e;
    if ((e = st.pull())) return e;
    for (int c = 0; c < n; ++c) {
      const double inv = ww[c] > 0 ? 1.0 / std::sqrt(ww[c]) : 0.0;
      if (!std::isfinite(inv)) return fail(LQ_ENUMERIC, "GCR: non-finite direction norm");
      st.h(c, ST_AUX) = inv;
      st.h(c, ST_AUX + 1) = 0.0;
    }
    if ((e = st.push())) return e;
    if ((e = bl.op(OP_SCALE, &wk, nullptr, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
        (e = bl.op(OP_SCALE, &zk, nullptr, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)))
      return e;
    // alpha = <w_k, r>: x += alpha z_k, r -= alpha w_k
    if ((e = bl.op(OP_DOT, &wk, &r)) || (e = to_aux())) return e;
    if ((e = bl.op(OP_AXPY, &zk, &x, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
        (e = bl.op(OP_AXMY, &wk, &r, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)))
      return e;
    if ((e = col_norms(bl, r, rr))) return e;
    ++it;
    ++k;
    if (verbose()) {
      double wr = 0.0;
      for (int c = 0; c < n; ++c) wr = std::max(wr, bb[c] > 0 ? std::sqrt(rr[c] / bb[c]) : 0.0);
      fprintf(stderr, "[lq] %s step %d (%d iterations so far): worst rel. residual %.3e\n", tag, it, cnt.iters, wr);
    }
  }
  if (steps) *steps = it;
  // final true residual
  if ((e = true_res()) || (e = col_norms(bl, r, rr))) return e;
  return converged() ? LQ_OK : LQ_ENOCONV;
}

// GCR preconditioned by a short sloppy BiCGStab solve of M z = r from zero
// (to inner_tol relative to r, at most inner_iters iterations); cnt.iters
// counts the inner iterations
int gcr_mixed(Blas& bl, const Geom& g, const OpFn& M_hi, const OpFn& M_lo, int plo, Vec& x, Vec& b,
              const std::vector<double>& tol_in, int maxiter, double delta, Counters& cnt, const FusedFn* M_fused,
              int kmax, double inner_tol, int inner_iters) {
  std::vector<double> inner_tolv(b.ncol, inner_tol);
  PrecFn K = [&](Vec& z, Vec& r, Counters& c) {
    int e = vec_zero(z);
    if (e) return e;
    Counters inner;
    const int ri = bicgstab_mixed(bl, g, M_hi, M_lo, plo, z, r, inner_tolv, inner_iters, delta, inner, M_fused);
    if (ri != LQ_OK && ri != LQ_ENOCONV) return ri;
    c.iters += inner.iters;
    return 0;
  };
  Counters outer;
  const int rs = fgcr(bl, g, M_hi, K, x, b, tol_in, maxiter, outer, kmax, "gcr");
  cnt.iters += outer.iters;
  cnt.reliable += outer.reliable;
  return rs;
}

// Flexible GCR with sloppy inner vectors: every cycle of kmax directions runs
// in precision plo (directions z_k = K(r), w_k = M z_k, their classical
// Gram-Schmidt against the earlier directions in one pass,
// the iterated residual and the cycle's correction), and ends with an FP64
// update: x += correction, then r = b - M x in FP64 starts the next cycle (a
// reliable update per cycle).  *steps counts the directions.  Three cycles
// in a row that reduce the worst true residual by less than 10% end the solve
// (LQ_ENOCONV).
int fgcr_mixed(Blas& bl, const Geom& g, const OpFn& M_hi, const OpFn& M_lo, const PrecFn& K, int plo, Vec& x,
               Vec& b, const std::vector<double>& tol, int maxiter, Counters& cnt, int kmax, const char* tag,
               int* steps) {
  const int n = b.ncol, nc = b.nc, npar = b.npar, par0 = b.par0;
  hipStream_t s = bl.s;
  Vec r = make_vec(g, 64, nc, n, npar, par0, s), q = make_vec(g, 64, nc, n, npar, par0, s);
  Vec rs = make_vec(g, plo, nc, n, npar, par0, s), xs = make_vec(g, plo, nc, n, npar, par0, s);
  std::vector<Vec> Z, W;
  for (int k = 0; k < kmax; ++k) {
    Z.push_back(make_vec(g, plo, nc, n, npar, par0, s));
    W.push_back(make_vec(g, plo, nc, n, npar, par0, s));
    if (!Z.back().ok() || !W.back().ok()) return fail(LQ_ENOMEM, "gcr buffers");
  }
  State st(n, s);
  DBuf cgs_part((size_t)8 * n * bl.gridx * 2 * sizeof(double), s), cgs_coef((size_t)8 * n * 2 * sizeof(double), s);
  if (!r.ok() || !q.ok() || !rs.ok() || !xs.ok() || !st.ok() || !cgs_part.p || !cgs_coef.p)
    return fail(LQ_ENOMEM, "gcr buffers");
  for (int c = 0; c < n; ++c) {
    for (int k = 0; k < ST_STRIDE; ++k) st.h(c, k) = 0.0;
    st.h(c, ST_ACTIVE) = 1.0;
  }
  int e = st.push();
  if (e) return e;
  std::vector<double> bb, rr;
  if ((e = col_norms(bl, b, bb))) return e;
  auto converged = [&]() -> bool {
    for (int c = 0; c < n; ++c)
      if (bb[c] > 0 && rr[c] > tol[c] * tol[c] * bb[c]) return false;
    return true;
  };
  auto to_aux = [&]() -> int {
    return launch_scalar(SC_DOT_TO_AUX, bl.partial, bl.gridx, n, st.d(), s) ? fail(LQ_EDEVICE, "scalar") : 0;
  };
  auto true_res = [&]() -> int {
    int rc = M_hi(q, x);
    if (!rc) rc = bl.op(OP_XMY_NORM, &b, &q);
    if (rc) return rc;
    std::swap(r, q);
    return col_norms(bl, r, rr);
  };
  auto worst = [&]() -> double {
    double w = 0.0;
    for (int c = 0; c < n; ++c) w = std::max(w, bb[c] > 0 ? rr[c] / bb[c] : 0.0);
    return w;
  };
  int it = 0, stalled = 0;
  if ((e = true_res())) return e;
  while (it < maxiter && !converged()) {
    const double before = worst();
    if ((e = vec_copy(rs, r)) || (e = vec_zero(xs))) return e;
    for (int k = 0; k < kmax && it < maxiter; ++k) {
      Vec& zk = Z[k];
      Vec& wk = W[k];
      if ((e = K(zk, rs, cnt)) || (e = M_lo(wk, zk))) return e;
      // classical Gram-Schmidt against the earlier directions, up to 8 in one pass
      for (int j0 = 0; j0 < k; j0 += 8) {
        FieldRef Wf[8], Zf[8];
        const int kk = std::min(8, k - j0);
        for (int j = 0; j < kk; ++j) {
          Wf[j] = W[j0 + j].f;
          Zf[j] = Z[j0 + j].f;
        }
        // algorithmic bytes: w and the W_j read for the dots, then W_j, Z_j read and w, z read and written
        const double vb = (double)wk.bytes > 0 ? (double)wk.bytes : (double)vec_bytes(g, plo, nc, n, npar);
        Prof pc(bl.ctx, "mg_cgs", s, vb * (3.0 * kk + 5.0));
        if (launch_mg_cgs(plo, Wf, Zf, kk, wk.f, zk.f, n, npar, bl.gridx, cgs_part.as<double>(),
                          cgs_coef.as<double>(), s))
          return fail(LQ_EDEVICE, "gram-schmidt");
      }
      std::vector<double> ww;
      if ((e = col_norms(bl, wk, ww)) || (e = st.pull())) return e;
      for (int c = 0; c < n; ++c) {
        const double inv = ww[c] > 0 ? 1.0 / std::sqrt(ww[c]) : 0.0;
        if (!std::isfinite(inv)) return fail(LQ_ENUMERIC, "GCR: non-finite direction norm");
        st.h(c, ST_AUX) = inv;
        st.h(c, ST_AUX + 1) = 0.0;
      }
      if ((e = st.push())) return e;
      if ((e = bl.op(OP_SCALE, &wk, nullptr, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
          (e = bl.op(OP_SCALE, &zk, nullptr, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)))
        return e;
      if ((e = bl.op(OP_DOT, &wk, &rs)) || (e = to_aux())) return e;
      if ((e = bl.op(OP_AXPY, &zk, &xs, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
          (e = bl.op(OP_AXMY, &wk, &rs, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
          (e = col_norms(bl, rs, rr)))
        return e;
      ++it;
      if (verbose()) {
        double wr = 0.0;
        for (int c = 0; c < n; ++c) wr = std::max(wr, bb[c] > 0 ? std::sqrt(rr[c] / bb[c]) : 0.0);
        fprintf(stderr, "[lq] %s step %d: worst iterated rel. residual %.3e\n", tag, it, wr);
      }
      if (converged()) break;
    }
    // the cycle's correction in FP64, then the true residual
    if (launch_axpy_mixed(x.f, 64, xs.f, plo, nc, n, npar, g.Vh, s)) return fail(LQ_EDEVICE, "axpy");
    ++cnt.reliable;
    if ((e = true_res())) return e;
    // three cycles in a row that reduce the worst true residual by less than 10% end the solve
    stalled = worst() > 0.81 * before ? stalled + 1 : 0;
    if (stalled >= 3) break;
  }
  if (steps) *steps = it;
  return converged() ? LQ_OK : LQ_ENOCONV;
}

// One two-level V-cycle in FP32 as the preconditioner of the outer GCR on the
// full-lattice D (sec. 2.1, Table 2's multigrid): restrict the residual, solve
// the even-odd preconditioned coarse system by BiCGStab (FP32 coarse operator,
// FP64 reliable updates, to coarse_tol), reconstruct and prolong, then smooth
// on the fine level: with r' = r - D e, nu_post minimal-residual steps on the
// even-odd system M_hat e_e = bhat_e(r') (t = residual, u = M_hat t with
// <u, t> and |u|^2 fused into the stencil, e_e += omega t, t -= omega u,
// omega = <u, t> / |u|^2 per column), then e += the reconstructed correction.
// With nu_pre > 0 the same smoother first acts on r, and the coarse level
// restricts r - D e_pre (e_pre is kept in the correction).
struct MgCycle {
  OpEnv& env;
  const MgHier& h;
  Blas& bl;  // fine-level reductions (full lattice)
  int n;
  Vec r32, e32, t32, bc, xc, be, xe, to, ue, tmp64, tmp32;
  Vec she, sre, sue, sto, sde;  // smoother: even correction, residual, M_hat residual; odd temporary; full correction
  Vec spre;                     // pre-smoothing correction (nu_pre > 0)
  Blas blc, ble;
  DBuf red;
  int tiles = 0;
  State st;
  Counters coarse;
  int cycles = 0;
  bool fp64_io = false;
  MgCycle(OpEnv& en, const MgHier& hh, Blas& b, int ncol) : env(en), h(hh), bl(b), n(ncol), st(ncol, en.s) {}
  int init() {
    const Geom& g = env.f->g;
    hipStream_t s = env.s;
    if (fp64_io) {  // conversion buffers for callers passing FP64 residuals and directions
      r32 = make_vec(g, 32, 12, n, 2, 0, s);
      e32 = make_vec(g, 32, 12, n, 2, 0, s);
    }
    t32 = make_vec(g, 32, 12, n, 2, 0, s);
    bc = make_vec(h.gc, 64, 12, n, 2, 0, s);
    xc = make_vec(h.gc, 64, 12, n, 2, 0, s);
    be = make_vec(h.gc, 64, 12, n, 1, 0, s);
    xe = make_vec(h.gc, 64, 12, n, 1, 0, s);
    ue = make_vec(h.gc, 64, 12, n, 1, 0, s);
    to = make_vec(h.gc, 64, 12, n, 1, 1, s);
    tmp64 = make_vec(h.gc, 64, 12, n, 1, 1, s);
    tmp32 = make_vec(h.gc, 32, 12, n, 1, 1, s);
    she = make_vec(g, 32, 12, n, 1, 0, s);
    sre = make_vec(g, 32, 12, n, 1, 0, s);
    sue = make_vec(g, 32, 12, n, 1, 0, s);
    sto = make_vec(g, 32, 12, n, 1, 1, s);
    sde = make_vec(g, 32, 12, n, 2, 0, s);
    if (h.nu_pre > 0) {
      spre = make_vec(g, 32, 12, n, 2, 0, s);
      if (!spre.ok()) return fail(LQ_ENOMEM, "multigrid cycle buffers");
    }
    tiles = (g.Vh + 63) / 64;
    red = DBuf(sizeof(double) * 4 * (size_t)tiles * n, s);
    if ((fp64_io && (!r32.ok() || !e32.ok())) || !t32.ok() || !bc.ok() || !xc.ok() || !be.ok() || !xe.ok() ||
        !ue.ok() || !to.ok() || !tmp64.ok() || !tmp32.ok() || !she.ok() || !sre.ok() || !sue.ok() || !sto.ok() ||
        !sde.ok() || !red.p || !st.ok())
      return fail(LQ_ENOMEM, "multigrid cycle buffers");
    for (int c = 0; c < n; ++c) {
      for (int k = 0; k < ST_STRIDE; ++k) st.h(c, k) = 0.0;
      st.h(c, ST_ACTIVE) = 1.0;
    }
    int e = st.push();
    if (!e) e = blas_prepare(env.ctx, blc, h.gc, 1, n, s);
    if (!e) e = blas_prepare(env.ctx, ble, g, 1, n, s);
    return e;
  }
  // sde = the correction of nu minimal-residual steps on the even-odd system
  // for the full-lattice residual res (zero start; res is left unchanged)
  int smooth(Vec& res, int nu) {
    int e = 0;
    if ((e = tm_schur_source(env, sre, res)) || (e = vec_zero(she))) return e;
    for (int k = 0; k < nu; ++k) {
      if ((e = tm_schur(env, 32, sue, sre, sto, 2, red.as<double>()))) return e;
      if (launch_scalar(SC_BICG_OMEGA, red.as<double>(), tiles, n, st.d(), env.s)) return fail(LQ_EDEVICE, "scalar");
      if ((e = ble.op(OP_AXPY, &sre, &she, nullptr, nullptr, nullptr, st.d(), ST_OMEGA, ST_OMEGA))) return e;
      if (k + 1 < nu && (e = ble.op(OP_AXMY, &sue, &sre, nullptr, nullptr, nullptr, st.d(), ST_OMEGA, ST_OMEGA)))
        return e;
    }
    return tm_schur_reconstruct(env, sde, she, res);
  }
  // z = K r; r and z in FP32 are used in place, FP64 ones are converted
  int operator()(Vec& z, Vec& r) {
    int e = 0;
    if ((r.prec != 32 || z.prec != 32) && !fp64_io) return fail(LQ_EINVAL, "multigrid cycle: FP32 vectors expected");
    if (r.prec != 32 && (e = vec_copy(r32, r))) return e;
    Vec& rin = r.prec == 32 ? r : r32;
    Vec& ev = z.prec == 32 ? z : e32;
    // optional pre-smoothing: its correction e_pre, and the coarse level sees r - D e_pre
    Vec* res = &rin;
    if (h.nu_pre > 0) {
      if ((e = smooth(rin, h.nu_pre)) || (e = vec_copy(spre, sde))) return e;
      if ((e = wilson_D(env, 32, t32, spre, false)) || (e = bl.op(OP_XMY_NORM, &rin, &t32))) return e;
      res = &t32;
    }
    // coarse solve on the even aggregates: (1 - A_ee^-1 D_eo A_oo^-1 D_oe) x_e = bhat_e
    if ((e = mg_restrict(env, h, *res, bc)) || (e = mg_schur_source(env, h, be, to, ue, bc)) || (e = vec_zero(xe)))
      return e;
    OpFn S = [&](Vec& o, const Vec& i) {
      Vec t = view(i.prec == 64 ? tmp64 : tmp32, 0, i.ncol);
      return mg_schur_op(env, h, o, i, t);
    };
    std::vector<double> tolc(n, h.coarse_tol);
    const int rc = bicgstab_mixed(blc, h.gc, S, S, 32, xe, be, tolc, h.coarse_maxiter, 0.1, coarse, nullptr);
    if (rc != LQ_OK && rc != LQ_ENOCONV) return rc;
    if ((e = mg_schur_reconstruct(env, h, xc, xe, to))) return e;
    if ((e = mg_prolong(env, h, xc, ev))) return e;
    if (h.nu_pre > 0 && (e = bl.opi(OP_AXPY, &spre, &ev, nullptr, 1.0))) return e;
    // fine-level smoothing on the residual of the correction so far, on the even-odd system
    if ((e = wilson_D(env, 32, t32, ev, false)) || (e = bl.op(OP_XMY_NORM, &rin, &t32))) return e;
    if ((e = smooth(t32, h.nu_post)) || (e = bl.opi(OP_AXPY, &sde, &ev, nullptr, 1.0))) return e;
    ++cycles;
    return z.prec == 32 ? 0 : vec_copy(z, e32);
  }
};

// near-null vectors for the multigrid setup: a few passes of inverse
// iteration w <- D^{-1} w / |D^{-1} w| from random vectors, each solve by the
// even-odd BiCGStab in FP32 with FP64 reliable updates
int mg_null_vectors(OpEnv& env, Vec& w, int passes, int maxiter, double tol, Counters& cnt) {
  const Geom& g = env.f->g;
  hipStream_t s = env.s;
  const int n = w.ncol;
  Vec x = make_vec(g, 64, 12, n, 2, 0, s);
  Vec bh = make_vec(g, 64, 12, n, 1, 0, s), xe = make_vec(g, 64, 12, n, 1, 0, s);
  Vec to64 = make_vec(g, 64, 12, n, 1, 1, s), to32 = make_vec(g, 32, 12, n, 1, 1, s);
  if (!x.ok() || !bh.ok() || !xe.ok() || !to64.ok() || !to32.ok()) return fail(LQ_ENOMEM, "multigrid setup buffers");
  Blas ble, bl;
  int e = blas_prepare(env.ctx, ble, g, 1, n, s);
  if (!e) e = blas_prepare(env.ctx, bl, g, 2, n, s);
  if (e) return e;
  OpFn M64 = [&](Vec& o, const Vec& i) { return tm_schur(env, 64, o, i, to64); };
  OpFn M32 = [&](Vec& o, const Vec& i) { return tm_schur(env, 32, o, i, to32); };
  FusedFn Mf = [&](Vec& o, const Vec& i, int mode, double* red) { return tm_schur(env, 32, o, i, to32, mode, red); };
  State st(n, s);
  if (!st.ok()) return fail(LQ_ENOMEM, "multigrid setup state");
  std::vector<double> tolv(n, tol), nn;
  for (int p = 0; p < passes; ++p) {
    if ((e = tm_schur_source(env, bh, w)) || (e = vec_zero(xe))) return e;
    const int rs = bicgstab_mixed(ble, g, M64, M32, 32, xe, bh, tolv, maxiter, 0.1, cnt, &Mf);
    if (rs != LQ_OK && rs != LQ_ENOCONV) return rs;
    if ((e = tm_schur_reconstruct(env, x, xe, w)) || (e = col_norms(bl, x, nn))) return e;
    for (int c = 0; c < n; ++c) {
      if (!(nn[c] > 0) || !std::isfinite(nn[c])) return fail(LQ_ENUMERIC, "multigrid setup: vanishing vector");
      for (int k = 0; k < ST_STRIDE; ++k) st.h(c, k) = 0.0;
      st.h(c, ST_AUX) = 1.0 / std::sqrt(nn[c]);
    }
    if ((e = st.push()) || (e = bl.op(OP_SCALE, &x, nullptr, nullptr, nullptr, nullptr, st.d(), ST_AUX, ST_AUX)) ||
        (e = vec_copy(w, x)))
      return e;
  }
  return 0;
}

}  // namespace

// ------------------------------------------------------------------ overlap
// Overlap propagators through the chirally projected normal equations
// (sec. 2.3).  With D = rho (1 + g5 eps) and eps^2 = 1, D is normal and
//   D^dag D = rho^2 (2 + g5 eps + eps g5)
// commutes with g5; on a vector of chirality s (g5 v = s v) it equals
// 2 rho^2 (v + s P_s eps v), P_s = (1 + s g5)/2: one sign function per
// application, and the result stays in the sector.  The massive operator
// D(m) = (1 - m/(2 rho)) D + m satisfies
//   D(m)^dag D(m) = (1 - m^2/(4 rho^2)) (H_s + sigma(m)),
//   H_s = D^dag D on the sector, sigma(m) = m^2 / (1 - m^2/(4 rho^2)),
// so all masses are shifts of one operator (multi-shift CG), and
// x(m) = D(m)^dag z(m) with D(m)^dag D(m) z(m) = b (normality).  A source is
// split into its two chiral halves; a point source has one.  With the
// polynomial sign function eps_N^2 differs from 1 by the approximation error,
// so the sector solve is wrapped in defect correction: the FP64 residual
// b - D(m) x is recomputed with the full operator and solved for again
// (both chiralities) until it meets the target.
namespace {

struct SecCol {
  int i, j, s;  // mass index (ascending order), source column, chirality
};

// p coefficients of OP_PLC for the operators used below
void plc_sector(double* q, double rho, double m, int s) {  // (1 - m^2/4rho^2)(H_s) + m^2
  const double f = 1.0 - m * m / (4.0 * rho * rho);
  q[0] = f * 2.0 * rho * rho + m * m;
  q[1] = f * rho * rho;
  q[2] = s;
  q[3] = 1.0;
}
void plc_shifted(double* q, double rho, double sigma, int s) {  // H_s + sigma
  q[0] = 2.0 * rho * rho + sigma;
  q[1] = rho * rho;
  q[2] = s;
  q[3] = 1.0;
}

}  // namespace

static int overlap_solve(OpEnv& env, const lq_params* prm, int n_rhs, const double* b_dev, double* x_dev,
                         double tol, int maxiter, double delta, int plo, Counters& cnt, double& worst, int& status) {
  lq_ctx* c = env.ctx;
  const Geom& g = env.f->g;
  hipStream_t s = env.s;
  const double rho = env.act.rho;
  int e = 0;
  if ((e = overlap_prepare(env))) return e;
  const int nm = prm->n_shift > 1 ? prm->n_shift : 1;
  std::vector<double> mass_in(nm, env.act.m);
  if (prm->n_shift > 1) {
    if (!prm->masses) return fail(LQ_EINVAL, "overlap multi-mass solve needs masses");
    mass_in.assign(prm->masses, prm->masses + nm);
  }
  for (double m : mass_in)
    if (!(m > 0) || !(m < 2 * rho)) return fail(LQ_EINVAL, "overlap masses must lie in (0, 2 rho)");
  if (prm->use_initial_guess && nm > 1) return fail(LQ_EINVAL, "overlap: initial guess with one mass only");
  // internal order: ascending mass (ascending sigma), so the base shift comes first
  std::vector<int> order(nm);
  for (int i = 0; i < nm; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return mass_in[a] < mass_in[b2]; });
  std::vector<double> mass(nm);
  for (int i = 0; i < nm; ++i) mass[i] = mass_in[order[i]];
  const int nx = nm * n_rhs;  // solution columns, mass-major

  Vec b = make_vec(g, 64, 12, n_rhs, 2, 0, s);
  Vec brep = make_vec(g, 64, 12, nx, 2, 0, s);
  Vec x = make_vec(g, 64, 12, nx, 2, 0, s);
  Vec r = make_vec(g, 64, 12, nx, 2, 0, s);
  Vec t1 = make_vec(g, 64, 12, nx, 2, 0, s);
  Vec t2 = make_vec(g, 64, 12, nx, 2, 0, s);
  DBuf pxd(sizeof(double) * 4 * nx, s), pxdag(sizeof(double) * 4 * nx, s);
  if (!b.ok() || !brep.ok() || !x.ok() || !r.ok() || !t1.ok() || !t2.ok() || !pxd.p || !pxdag.p)
    return fail(LQ_ENOMEM, "overlap solution buffers");
  if (launch_pack_field(g, b_dev, n_rhs, 12, b.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
  for (int i = 0; i < nm; ++i)
    if (launch_convert(brep.cols(i * n_rhs), 64, b.f, 64, 12, n_rhs, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
  if (prm->use_initial_guess) {
    if (launch_pack_field(g, x_dev, n_rhs, 12, x.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
  } else if ((e = vec_zero(x))) return e;
  // D(m) v = (rho + m/2) v + (rho - m/2) g5 eps v ; D(m)^dag v = (rho + m/2) v + (rho - m/2) eps g5 v
  {
    std::vector<double> hd((size_t)4 * nx), hdag((size_t)4 * nx);
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < n_rhs; ++j) {
        double* q = &hd[(size_t)4 * (i * n_rhs + j)];
        double* qd = &hdag[(size_t)4 * (i * n_rhs + j)];
        q[0] = qd[0] = rho + 0.5 * mass[i];
        q[1] = qd[1] = rho - 0.5 * mass[i];
        q[2] = 0.0; q[3] = 1.0;
        qd[2] = 1.0; qd[3] = 0.0;
      }
    hipMemcpyAsync(pxd.p, hd.data(), sizeof(double) * hd.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(pxdag.p, hdag.data(), sizeof(double) * hdag.size(), hipMemcpyHostToDevice, s);
  }
  Blas bl;
  if ((e = blas_prepare(c, bl, g, 2, 2 * nx, s))) return e;
  std::vector<double> bb;
  if ((e = col_norms(bl, b, bb))) return e;

  // r = brep - D(m) x on every solution column; res = |r| / |b|
  std::vector<double> res(nx, 1.0);
  auto residual = [&]() -> int {
    int rr = 0;
    if ((rr = sign_apply(env, 64, t1, x))) return rr;
    if ((rr = bl.plc(&x, &t1, &r, pxd.as<double>()))) return rr;
    if ((rr = bl.op(OP_XMY_NORM, &brep, &r))) return rr;  // r = brep - D x
    State st(nx, s);
    if (!st.ok()) return fail(LQ_ENOMEM, "state");
    if (launch_scalar(SC_SET_RR, bl.partial, bl.gridx, nx, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if ((rr = st.pull())) return rr;
    for (int k = 0; k < nx; ++k) {
      const double bk = bb[k % n_rhs];
      res[k] = bk > 0 ? std::sqrt(st.h(k, ST_RR) / bk) : 0.0;
      if (!std::isfinite(res[k])) return fail(LQ_ENUMERIC, "NaN/Inf in the overlap residual");
    }
    return 0;
  };

  const int pms = plo == 16 ? 32 : plo;  // precision of the multi-shift stage
  bool have_r = false;                   // r holds the residual of x
  if (prm->use_initial_guess) {
    if ((e = residual())) return e;
    have_r = true;
  }
  worst = 1.0;
  status = LQ_OK;
  for (int pass = 0; pass < 8; ++pass) {
    if (have_r) {
      worst = *std::max_element(res.begin(), res.end());
      if (worst <= tol) break;
    }
    // chiral sector sources: pass 0 from b (shared by the masses), later passes
    // from the residual of each unconverged (mass, column)
    std::vector<double> nrm;
    Vec src = make_vec(g, 64, 12, have_r ? nx : n_rhs, 2, 0, s);
    if (!src.ok()) return fail(LQ_ENOMEM, "overlap sector buffers");
    if ((e = vec_copy(src, have_r ? r : b))) return e;
    std::vector<SecCol> cols;
    {
      Vec halves = make_vec(g, 64, 12, 2 * src.ncol, 2, 0, s);
      DBuf pp(sizeof(double) * 8 * src.ncol, s);
      if (!halves.ok() || !pp.p) return fail(LQ_ENOMEM, "overlap sector buffers");
      std::vector<double> hp((size_t)8 * src.ncol);
      for (int k = 0; k < 2 * src.ncol; ++k) {
        const int sg = (k & 1) ? -1 : 1;
        double* q = &hp[(size_t)4 * k];
        q[0] = 0.0; q[1] = 0.5; q[2] = 1.0; q[3] = sg;  // P_s v = (v + s g5 v) / 2
        if (launch_convert(halves.cols(k), 64, src.cols(k / 2), 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      }
      hipMemcpyAsync(pp.p, hp.data(), sizeof(double) * hp.size(), hipMemcpyHostToDevice, s);
      if ((e = bl.plc(&halves, &halves, &halves, pp.as<double>()))) return e;
      if ((e = col_norms(bl, halves, nrm))) return e;
      // keep the nonzero halves (of unconverged columns)
      std::vector<int> keep;
      for (int k = 0; k < 2 * src.ncol; ++k) {
        const int sc = k / 2;
        if (have_r && res[sc] <= tol) continue;
        if (!(nrm[k] > 0)) continue;
        keep.push_back(k);
      }
      if (!have_r) {
        // pass 0: the same sector sources for every mass, mass-major
        for (int i = 0; i < nm; ++i)
          for (int k : keep) cols.push_back(SecCol{i, k / 2, (k & 1) ? -1 : 1});
      } else {
        for (int k : keep) cols.push_back(SecCol{(k / 2) / n_rhs, (k / 2) % n_rhs, (k & 1) ? -1 : 1});
      }
      const int ncs = (int)cols.size();
      if (ncs == 0) {
        if (!have_r) {  // b = 0: x = 0
          worst = 0.0;
          std::fill(res.begin(), res.end(), 0.0);
          break;
        }
        break;
      }
      src = make_vec(g, 64, 12, ncs, 2, 0, s);
      if (!src.ok()) return fail(LQ_ENOMEM, "overlap sector buffers");
      const int nkeep = (int)keep.size();
      for (int q = 0; q < ncs; ++q) {
        const int k = have_r ? keep[q] : keep[q % nkeep];
        if (launch_convert(src.cols(q), 64, halves.cols(k), 64, 12, 1, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      }
    }
    const int ncs = src.ncol;
    Vec z = make_vec(g, 64, 12, ncs, 2, 0, s);
    if (!z.ok()) return fail(LQ_ENOMEM, "overlap sector buffers");
    if ((e = vec_zero(z))) return e;
    ColParam cp;
    cp.stride = 4;
    cp.s = s;
    cp.host.assign((size_t)4 * ncs, 0.0);
    for (int q = 0; q < ncs; ++q) plc_sector(&cp.host[(size_t)4 * q], rho, mass[cols[q].i], cols[q].s);
    DBuf dcp(sizeof(double) * cp.host.size(), s);
    if (!dcp.p) return fail(LQ_ENOMEM, "overlap parameters");
    cp.dev = dcp.as<double>();
    if ((e = cp.upload())) return e;

    if (!have_r && nm > 1) {
      // multi-shift CG on H_s + sigma_i (sloppy, no reliable updates), base = lightest mass
      const int nsec = ncs / nm;
      std::vector<double> sig(nm);
      for (int i = 0; i < nm; ++i) sig[i] = mass[i] * mass[i] / (1.0 - mass[i] * mass[i] / (4.0 * rho * rho));
      std::vector<double> dsh(nm);
      for (int i = 0; i < nm; ++i) dsh[i] = sig[i] - sig[0];
      DBuf dsig(sizeof(double) * nm, s), pbase(sizeof(double) * 4 * nsec, s);
      Vec rr = make_vec(g, pms, 12, nsec, 2, 0, s), ap = make_vec(g, pms, 12, nsec, 2, 0, s),
          ee = make_vec(g, pms, 12, nsec, 2, 0, s), p = make_vec(g, pms, 12, ncs, 2, 0, s),
          xm = make_vec(g, pms, 12, ncs, 2, 0, s);
      State st(nsec, s);
      DBuf sh(sizeof(double) * 8 * ncs, s);
      if (!dsig.p || !pbase.p || !rr.ok() || !ap.ok() || !ee.ok() || !p.ok() || !xm.ok() || !st.ok() || !sh.p)
        return fail(LQ_ENOMEM, "overlap multi-shift buffers");
      hipMemcpyAsync(dsig.p, dsh.data(), sizeof(double) * nm, hipMemcpyHostToDevice, s);
      {
        std::vector<double> hb((size_t)4 * nsec);
        for (int q = 0; q < nsec; ++q) plc_shifted(&hb[(size_t)4 * q], rho, sig[0], cols[q].s);
        hipMemcpyAsync(pbase.p, hb.data(), sizeof(double) * hb.size(), hipMemcpyHostToDevice, s);
      }
      Vec src0 = view(src, 0, nsec);
      if (vec_copy(rr, src0) || vec_zero(xm)) return fail(LQ_EDEVICE, "init");
      for (int i = 0; i < nm; ++i)
        if (launch_convert(p.cols(i * nsec), pms, src0.f, 64, 12, nsec, 2, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      const double tol_ms = std::max(tol, pms == 32 ? 1e-6 : pms == 16 ? 2e-3 : tol);
      for (int j = 0; j < nsec; ++j) {
        for (int k = 0; k < ST_STRIDE; ++k) st.h(j, k) = 0.0;
        st.h(j, ST_ACTIVE) = 1.0;
        st.h(j, ST_PAD) = tol_ms * tol_ms;
      }
      if ((e = st.push())) return e;
      Blas blr;
      if ((e = blas_prepare(c, blr, g, 2, ncs, s))) return e;
      MsArgs M{};
      M.prec = pms; M.nc = 12; M.nrhs = nsec; M.nshift = nm; M.npar = 2; M.Vh = g.Vh;
      M.x = xm.f; M.p = p.f; M.r = rr.f; M.ap = ap.f;
      M.sh = sh.as<double>(); M.st = st.d(); M.partial = blr.partial; M.gridx = blr.gridx;
      if ((e = blr.op(OP_NORM2, &rr))) return e;
      if (launch_ms_init(M, s)) return fail(LQ_EDEVICE, "ms init");
      std::vector<double> hsh((size_t)8 * ncs);
      Vec p0 = view(p, 0, nsec);
      int it = 0;
      for (; it < maxiter; ++it) {
        if ((e = sign_apply(env, pms, ee, p0))) return e;
        if ((e = blr.plc(&p0, &ee, &ap, pbase.as<double>()))) return e;
        if ((e = blr.op(OP_DOT, &p0, &ap))) return e;
        if (launch_ms_scalar_alpha(M, dsig.as<double>(), s)) return fail(LQ_EDEVICE, "ms alpha");
        {
          MsProf pr(c, M, false, s);
          if (launch_ms_xr(M, s)) return fail(LQ_EDEVICE, "ms xr");
        }
        if (launch_ms_scalar_beta(M, s)) return fail(LQ_EDEVICE, "ms beta");
        {
          MsProf pr(c, M, true, s);
          if (launch_ms_p(M, s)) return fail(LQ_EDEVICE, "ms p");
        }
        hipMemcpyAsync(hsh.data(), sh.p, sizeof(double) * 8 * ncs, hipMemcpyDeviceToHost, s);
        if ((e = st.pull())) return e;
        bool any = false;
        for (int k = 0; k < ncs; ++k) any |= hsh[(size_t)k * 8 + 4] != 0.0;
        for (int j = 0; j < nsec; ++j)
          if (st.h(j, ST_FLAG) == 2.0) return fail(LQ_ENUMERIC, "NaN/Inf in multi-shift CG");
        if (!any) break;
      }
      cnt.iters += it;
      // z_i = (H_s + sigma_i)^{-1} src / (1 - m_i^2 / (4 rho^2))
      if ((e = vec_copy(z, xm))) return e;
      for (int i = 0; i < nm; ++i) {
        Vec zi = view(z, i * nsec, nsec);
        if ((e = bl.opi(OP_SCALE, &zi, nullptr, nullptr, 1.0 / (1.0 - mass[i] * mass[i] / (4.0 * rho * rho)))))
          return e;
      }
    }

    // deflation: the initial guess from the resident low modes of each column's
    // chiral sector, z0 = sum_i u_i <u_i, src> / (f mu_i + m^2), for the columns
    // that do not start from the multi-shift solution
    const bool from_ms = !have_r && nm > 1;
    if (prm->deflate > 0 && !from_ms) {
      for (int q = 0; q < ncs; ++q) {
        const EigSet* es = find_eigs(env.f, LQ_EIG_OVERLAP, rho, cols[q].s);
        if (!es || es->n < prm->deflate)
          return fail(LQ_EINVAL, "overlap: deflate needs that many resident sector modes (lq_eigs LQ_EIG_OVERLAP)");
        const int nd = prm->deflate;
        const double mq = mass[cols[q].i], fq = 1.0 - mq * mq / (4.0 * rho * rho);
        Vec sq = make_vec(g, 64, 12, 1, 2, 0, s), zq = view(z, q, 1);
        DBuf cf(sizeof(double) * 2 * nd, s);
        if (!sq.ok() || !cf.p) return fail(LQ_ENOMEM, "deflation buffers");
        Vec srcq = view(src, q, 1);
        if ((e = vec_copy(sq, srcq)) || (e = project_out(c, g, s, *es, nd, sq, cf.p))) return e;
        std::vector<double> wts(nd);
        for (int i = 0; i < nd; ++i) wts[i] = 1.0 / (fq * es->vals[i] + mq * mq);
        if ((e = vec_zero(zq)) || (e = add_modes(c, g, s, *es, nd, wts, zq, cf.p))) return e;
      }
    }

    // sector solve with FP64 reliable updates (the sector operator per column)
    Vec e64 = make_vec(g, 64, 12, ncs, 2, 0, s), elo = make_vec(g, plo, 12, ncs, 2, 0, s);
    if (!e64.ok() || !elo.ok()) return fail(LQ_ENOMEM, "overlap sector buffers");
    Blas bls;
    if ((e = blas_prepare(c, bls, g, 2, ncs, s))) return e;
    OpFn Ahi = [&](Vec& o, const Vec& in) {
      Vec t = view(e64, 0, in.ncol);
      int rr = sign_apply(env, 64, t, in);
      return rr ? rr : bls.plc(const_cast<Vec*>(&in), &t, &o, cp.dev);
    };
    OpFn Alo = [&](Vec& o, const Vec& in) {
      Vec t = view(elo, 0, in.ncol);
      int rr = sign_apply(env, plo, t, in);
      return rr ? rr : bls.plc(const_cast<Vec*>(&in), &t, &o, cp.dev);
    };
    // |r_ij - D D^dag z| <= tol |b_j| from per-sector targets relative to each sector source
    std::vector<double> tolv(ncs);
    {
      std::vector<double> sn;
      if ((e = col_norms(bl, src, sn))) return e;
      for (int q = 0; q < ncs; ++q) {
        const double bj = std::sqrt(bb[cols[q].j]), sq = std::sqrt(sn[q]);
        tolv[q] = sq > 0 ? std::min(0.1, 0.25 * tol * bj / sq) : 1.0;
      }
    }
    const int rs = cg_mixed(bls, g, Ahi, Alo, plo, z, src, tolv, maxiter, delta, cnt, &cp);
    if (rs != LQ_OK && rs != LQ_ENOCONV) return rs;
    status = rs;
    // y_ij = sum of the sector solutions ; x_ij += D(m_i)^dag y_ij
    if ((e = vec_zero(t2))) return e;
    for (int q = 0; q < ncs; ++q) {
      const int col = cols[q].i * n_rhs + cols[q].j;
      Vec zq = view(z, q, 1), yq = view(t2, col, 1);
      if ((e = bl.opi(OP_AXPY, &zq, &yq, nullptr, 1.0))) return e;
    }
    if ((e = bl.op(OP_G5, &t2, &r))) return e;
    if ((e = sign_apply(env, 64, t1, r))) return e;
    if ((e = bl.plc(&t2, &t1, &r, pxdag.as<double>()))) return e;
    if ((e = bl.opi(OP_AXPY, &r, &x, nullptr, 1.0))) return e;
    if ((e = residual())) return e;
    have_r = true;
    worst = *std::max_element(res.begin(), res.end());
    if (verbose())
      fprintf(stderr, "[lq] overlap pass %d: %d sector columns, worst rel. residual of D(m) x = b %.3e\n", pass, ncs,
              worst);
    if (worst <= tol || rs == LQ_ENOCONV) break;
  }
  // output in the caller's mass order: x is [n_shift][n_rhs][V][4][3]
  const size_t colsz = (size_t)2 * g.Vh * 12 * 2;
  for (int i = 0; i < nm; ++i) {
    Vec v = view(x, i * n_rhs, n_rhs);
    if (launch_unpack_field(g, v.f, 64, n_rhs, 12, x_dev + (size_t)order[i] * n_rhs * colsz, 2, s))
      return fail(LQ_EDEVICE, "unpack");
  }
  return 0;
}

// ------------------------------------------------------------------ top-level solve
int solve(lq_ctx* c, const lq_action* act, lq_field* f, const lq_params* prm, int n_rhs, const double* b_dev,
          double* x_dev, lq_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const Geom& g = f->g;
  OpEnv env{c, f, *act, s};
  env.recon = prm->recon12;
  const double tol = prm->tol > 0 ? prm->tol : 1e-10;
  int maxiter = prm->maxiter > 0 ? prm->maxiter : 10000;
  const double delta = prm->reliable_delta > 0 ? prm->reliable_delta : 0.1;
  const int plo = prm->sloppy_bits == 16 ? 16 : prm->sloppy_bits == 32 ? 32 : 64;
  Counters cnt;
  cnt.fault = prm->fault_inject;
  if (prm->fault_inject == 2) return fail(LQ_ENOMEM, "injected allocation failure");
  if (prm->fault_inject == 3) maxiter = 1;
  Blas bl;
  int e = 0;
  double worst = 0.0;
  int status = LQ_OK;
  const int kind = act->kind;

  if (kind == LQ_OVERLAP && prm->solver != 1) {
    if (f->type != 0) return fail(LQ_EINVAL, "field type does not match the action");
    if ((e = overlap_solve(env, prm, n_rhs, b_dev, x_dev, tol, maxiter, delta, plo, cnt, worst, status))) return e;
  } else if (kind == LQ_WILSON || kind == LQ_TM_CLOVER || kind == LQ_OVERLAP) {
    if (kind == LQ_TM_CLOVER && plo == 16) return fail(LQ_ENOTSUP, "twisted-clover sloppy storage is FP32 or FP64");
    if (kind == LQ_OVERLAP && (e = overlap_prepare(env))) return e;
    Vec b = make_vec(g, 64, 12, n_rhs, 2, 0, s);
    Vec x = make_vec(g, 64, 12, n_rhs, 2, 0, s);
    if (!b.ok() || !x.ok()) return fail(LQ_ENOMEM, "solution buffers");
    if (launch_pack_field(g, b_dev, n_rhs, 12, b.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
    if (prm->use_initial_guess) {
      if (launch_pack_field(g, x_dev, n_rhs, 12, x.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
    } else if ((e = vec_zero(x))) return e;
    if ((e = blas_prepare(c, bl, g, 2, n_rhs, s))) return e;
    OpFn D64 = [&](Vec& o, const Vec& i) {
      if (kind == LQ_OVERLAP) return overlap_D(env, 64, o, i, false);
      return wilson_D(env, 64, o, i, false);
    };
    std::vector<double> res;
    if (prm->solver == 3) {
      // flexible GCR on the full lattice, one multigrid V-cycle per direction
      MgHier* h = f->mg;
      if (!mg_matches(h, act)) return fail(LQ_EINVAL, "solver 3 needs lq_mg_setup for this action on this field");
      if (prm->maxiter <= 0) maxiter = 1000;  // outer steps, each one V-cycle
      MgCycle K(env, *h, bl, n_rhs);
      if ((e = K.init())) return e;
      PrecFn P = [&](Vec& z, Vec& r, Counters&) { return K(z, r); };
      OpFn D32 = [&](Vec& o, const Vec& i) { return wilson_D(env, 32, o, i, false); };
      std::vector<double> tol_v(n_rhs, 0.5 * tol);
      for (int pass = 0; pass < 4; ++pass) {
        int steps = 0;
        const int rs = fgcr_mixed(bl, g, D64, D32, P, 32, x, b, tol_v, maxiter, cnt, h->gcr_kmax, "mg-gcr", &steps);
        if (rs != LQ_OK && rs != LQ_ENOCONV) return rs;
        cnt.iters += steps;
        if ((e = rel_residual(bl, D64, x, b, res, g))) return e;
        worst = *std::max_element(res.begin(), res.end());
        status = rs;
        if (verbose())
          fprintf(stderr, "[lq] multigrid solve: %d outer steps, %d coarse iterations, residual %.3e\n", steps,
                  K.coarse.iters, worst);
        if (worst <= tol || rs == LQ_ENOCONV) break;
        for (int k = 0; k < n_rhs; ++k)
          if (res[k] > tol) tol_v[k] *= std::max(0.05, 0.5 * tol / res[k]);
      }
    } else if (kind == LQ_TM_CLOVER && prm->solver != 1) {
      Vec bh = make_vec(g, 64, 12, n_rhs, 1, 0, s);
      Vec xe = make_vec(g, 64, 12, n_rhs, 1, 0, s);
      Vec to64 = make_vec(g, 64, 12, n_rhs, 1, 1, s);
      Vec tolo = make_vec(g, plo, 12, n_rhs, 1, 1, s);
      if (!bh.ok() || !xe.ok() || !to64.ok() || !tolo.ok()) return fail(LQ_ENOMEM, "schur buffers");
      if ((e = tm_schur_source(env, bh, b))) return e;
      // initial guess: even part of x
      if (prm->use_initial_guess) {
        // x.f blocks are [col][par]: take parity 0 of each column
        for (int col = 0; col < n_rhs; ++col) {
          FieldRef dst = xe.cols(col), src = x.cols(col);
          if (launch_convert(dst, 64, src, 64, 12, 1, 1, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
        }
      } else if ((e = vec_zero(xe))) return e;
      Blas ble;
      if ((e = blas_prepare(c, ble, g, 1, n_rhs, s))) return e;
      OpFn M64 = [&](Vec& o, const Vec& i) { return tm_schur(env, 64, o, i, to64); };
      OpFn Mlo = [&](Vec& o, const Vec& i) { return tm_schur(env, plo, o, i, tolo); };
      FusedFn Mfused = [&](Vec& o, const Vec& i, int mode, double* red) {
        return tm_schur(env, plo, o, i, tolo, mode, red);
      };
      const bool fuse = getenv("LQ_NO_FUSED_REDUCTIONS") == nullptr;
      std::vector<double> tol_s(n_rhs, 0.5 * tol);
      for (int pass = 0; pass < 6; ++pass) {
        const int rs = prm->solver == 2
                           ? gcr_mixed(ble, g, M64, Mlo, plo, xe, bh, tol_s, maxiter, delta, cnt,
                                       fuse ? &Mfused : nullptr, 8, 0.1, 50)
                           : bicgstab_mixed(ble, g, M64, Mlo, plo, xe, bh, tol_s, maxiter, delta, cnt,
                                            fuse ? &Mfused : nullptr);
        if (rs != LQ_OK && rs != LQ_ENOCONV) return rs;
        if ((e = tm_schur_reconstruct(env, x, xe, b))) return e;
        if ((e = rel_residual(bl, D64, x, b, res, g))) return e;
        worst = *std::max_element(res.begin(), res.end());
        status = rs;
        if (worst <= tol || rs == LQ_ENOCONV) break;
        for (int k = 0; k < n_rhs; ++k)
          if (res[k] > tol) tol_s[k] *= std::max(0.05, 0.5 * tol / res[k]);
      }
    } else {
      // CG on the normal equations D^dag D x = D^dag b
      OpFn Ddag64 = [&](Vec& o, const Vec& i) {
        if (kind == LQ_OVERLAP) return overlap_D(env, 64, o, i, true);
        return wilson_D(env, 64, o, i, true);
      };
      Vec tmp64 = make_vec(g, 64, 12, n_rhs, 2, 0, s);
      Vec tmplo = make_vec(g, plo, 12, n_rhs, 2, 0, s);
      Vec bn = make_vec(g, 64, 12, n_rhs, 2, 0, s);
      if (!tmp64.ok() || !tmplo.ok() || !bn.ok()) return fail(LQ_ENOMEM, "cgne buffers");
      if ((e = Ddag64(bn, b))) return e;
      // the solver passes views of its active columns: temporaries of the same width
      OpFn N64 = [&](Vec& o, const Vec& i) {
        Vec t = view(tmp64, 0, i.ncol);
        int r = D64(t, i);
        return r ? r : Ddag64(o, t);
      };
      OpFn Nlo = [&](Vec& o, const Vec& i) {
        Vec t = view(tmplo, 0, i.ncol);
        int r = kind == LQ_OVERLAP ? overlap_D(env, plo, t, i, false) : wilson_D(env, plo, t, i, false);
        if (r) return r;
        return kind == LQ_OVERLAP ? overlap_D(env, plo, o, t, true) : wilson_D(env, plo, o, t, true);
      };
      std::vector<double> tol_n(n_rhs, 0.1 * tol);
      for (int pass = 0; pass < 6; ++pass) {
        const int rs = cg_mixed(bl, g, N64, Nlo, plo, x, bn, tol_n, maxiter, delta, cnt);
        if (rs != LQ_OK && rs != LQ_ENOCONV) return rs;
        if ((e = rel_residual(bl, D64, x, b, res, g))) return e;
        worst = *std::max_element(res.begin(), res.end());
        status = rs;
        if (worst <= tol || rs == LQ_ENOCONV) break;
        for (int k = 0; k < n_rhs; ++k)
          if (res[k] > tol) tol_n[k] *= std::max(0.01, 0.5 * tol / res[k]);
      }
    }
    if (launch_unpack_field(g, x.f, 64, n_rhs, 12, x_dev, 2, s)) return fail(LQ_EDEVICE, "unpack");
  } else if (kind == LQ_HISQ) {
    const int nsh = prm->n_shift > 1 ? prm->n_shift : 1;
    std::vector<double> masses(nsh, act->m);
    if (prm->n_shift > 1) {
      if (!prm->masses) return fail(LQ_EINVAL, "HISQ multi-shift needs masses");
      masses.assign(prm->masses, prm->masses + nsh);
    }
    for (double m : masses)
      if (!(m > 0)) return fail(LQ_EINVAL, "HISQ masses must be positive");
    const int i0 = (int)(std::min_element(masses.begin(), masses.end()) - masses.begin());
    const double m0 = masses[i0];
    // shift order: base (smallest mass) first
    std::vector<int> order;
    order.push_back(i0);
    for (int i = 0; i < nsh; ++i)
      if (i != i0) order.push_back(i);
    std::vector<double> sigma(nsh), m2col((size_t)nsh * n_rhs), mcol((size_t)nsh * n_rhs);
    for (int k = 0; k < nsh; ++k) sigma[k] = masses[order[k]] * masses[order[k]] - m0 * m0;
    for (int k = 0; k < nsh; ++k)
      for (int j = 0; j < n_rhs; ++j) {
        m2col[(size_t)k * n_rhs + j] = masses[order[k]] * masses[order[k]];
        mcol[(size_t)k * n_rhs + j] = masses[order[k]];
      }
    const int ncol = nsh * n_rhs;
    DBuf dsig(sizeof(double) * nsh, s), dm2(sizeof(double) * ncol, s), dm(sizeof(double) * ncol, s);
    if (!dsig.p || !dm2.p || !dm.p) return fail(LQ_ENOMEM, "shift arrays");
    hipMemcpyAsync(dsig.p, sigma.data(), sizeof(double) * nsh, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dm2.p, m2col.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dm.p, mcol.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, s);
    Vec be = make_vec(g, 64, 3, n_rhs, 1, 0, s);
    Vec brep = make_vec(g, 64, 3, ncol, 1, 0, s);
    Vec y = make_vec(g, 64, 3, ncol, 1, 0, s);
    if (!be.ok() || !brep.ok() || !y.ok()) return fail(LQ_ENOMEM, "HISQ buffers");
    if (launch_pack_field(g, b_dev, n_rhs, 3, be.f, 64, 0, s)) return fail(LQ_EDEVICE, "pack");
    for (int k = 0; k < nsh; ++k)
      if (launch_convert(brep.cols(k * n_rhs), 64, be.f, 64, 3, n_rhs, 1, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
    Blas ble;
    if ((e = blas_prepare(c, ble, g, 1, ncol, s))) return e;
    if ((e = vec_zero(y))) return e;
    if (prm->use_initial_guess) {
      for (int k = 0; k < nsh; ++k) {
        Vec tmp = make_vec(g, 64, 3, n_rhs, 1, 0, s);
        if (launch_pack_field(g, x_dev + (size_t)order[k] * n_rhs * 2 * g.Vh * 3 * 2, n_rhs, 3, tmp.f, 64, 0, s))
          return fail(LQ_EDEVICE, "pack");
        if (launch_convert(y.cols(k * n_rhs), 64, tmp.f, 64, 3, n_rhs, 1, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      }
    } else if (nsh > 1) {
      // multi-shift CG, one Krylov space for all masses, to a loose tolerance
      // (it has no reliable updates, so it stops where its precision does).
      // With FP16 sloppy storage it runs in FP32: the shifted solutions then
      // start the FP16 refinement near 1e-8 instead of 2e-3, which moves work
      // from the refinement (an operator over every shift and column) to the
      // multi-shift iteration (an operator over the base columns only).  At
      // 32^3 x 96 with 8 masses the FP32 target 1e-8 measured best (4.0 s per
      // solve against 6.5 s for FP16 to 2e-3, 5.7 s for 1e-5, 4.8 s for 1e-6
      // and 1e-7, 4.5 s for 1e-9).
      const int pms = plo == 16 ? LQ_MS_PREC16 : plo;
      Vec r = make_vec(g, pms, 3, n_rhs, 1, 0, s);
      Vec ap = make_vec(g, pms, 3, n_rhs, 1, 0, s);
      Vec to = make_vec(g, pms, 3, n_rhs, 1, 1, s);
      Vec p = make_vec(g, pms, 3, ncol, 1, 0, s);
      Vec xm = make_vec(g, pms, 3, ncol, 1, 0, s);
      State st(n_rhs, s);
      DBuf sh(sizeof(double) * 8 * ncol, s);
      if (!r.ok() || !ap.ok() || !to.ok() || !p.ok() || !xm.ok() || !st.ok() || !sh.p)
        return fail(LQ_ENOMEM, "multi-shift buffers");
      if (vec_copy(r, be) || vec_zero(xm)) return fail(LQ_EDEVICE, "init");
      for (int k = 0; k < nsh; ++k)
        if (launch_convert(p.cols(k * n_rhs), pms, be.f, 64, 3, n_rhs, 1, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      const double tol_ms = std::max(tol, pms == 16 ? 2e-3 : pms == 32 ? LQ_MS_TOL32 : tol);
      for (int j = 0; j < n_rhs; ++j) {
        for (int k = 0; k < ST_STRIDE; ++k) st.h(j, k) = 0.0;
        st.h(j, ST_ACTIVE) = 1.0;
        st.h(j, ST_PAD) = tol_ms * tol_ms;
      }
      if ((e = st.push())) return e;
      Blas blr;
      if ((e = blas_prepare(c, blr, g, 1, ncol, s))) return e;
      MsArgs M{};
      M.prec = pms; M.nc = 3; M.nrhs = n_rhs; M.nshift = nsh; M.npar = 1; M.Vh = g.Vh;
      M.x = xm.f; M.p = p.f; M.r = r.f; M.ap = ap.f;
      M.sh = sh.as<double>(); M.st = st.d(); M.partial = blr.partial; M.gridx = blr.gridx;
      if ((e = blr.op(OP_NORM2, &r))) return e;
      if (launch_ms_init(M, s)) return fail(LQ_EDEVICE, "ms init");
      std::vector<double> hsh((size_t)8 * ncol);
      Vec p0 = view(p, 0, n_rhs);
      // <p_0, A p_0> from the stencil epilogue: partials over 64-site tiles
      const int mtiles = (g.Vh + 63) / 64;
      DBuf mred(sizeof(double) * 4 * (size_t)mtiles * n_rhs, s);
      if (!mred.p) return fail(LQ_ENOMEM, "multi-shift partials");
      MsArgs Ma = M;
      Ma.partial = mred.as<double>();
      Ma.gridx = mtiles;
      int it = 0;
      for (; it < maxiter; ++it) {
        if ((e = stag_normal_even(env, pms, ap, p0, to, nullptr, m0 * m0, mred.as<double>()))) return e;
        if (launch_ms_scalar_alpha(Ma, dsig.as<double>(), s)) return fail(LQ_EDEVICE, "ms alpha");
        {
          MsProf pr(c, M, false, s);
          if (launch_ms_xr(M, s)) return fail(LQ_EDEVICE, "ms xr");
        }
        if (launch_ms_scalar_beta(M, s)) return fail(LQ_EDEVICE, "ms beta");
        {
          MsProf pr(c, M, true, s);
          if (launch_ms_p(M, s)) return fail(LQ_EDEVICE, "ms p");
        }
        if ((it & 3) == 3 || it < 4) {
          hipMemcpyAsync(hsh.data(), sh.p, sizeof(double) * 8 * ncol, hipMemcpyDeviceToHost, s);
          if ((e = st.pull())) return e;
          bool any = false;
          for (int k = 0; k < ncol; ++k) any |= hsh[(size_t)k * 8 + 4] != 0.0;
          for (int j = 0; j < n_rhs; ++j)
            if (st.h(j, ST_FLAG) == 2.0) return fail(LQ_ENUMERIC, "NaN/Inf in multi-shift CG");
          if (!any) break;
        }
      }
      cnt.iters += it;
      if ((e = vec_copy(y, xm))) return e;
    }
    // per-shift mixed-precision CG refinement on M_e(m_i) (all shifts and columns batched)
    Vec to64 = make_vec(g, 64, 3, ncol, 1, 1, s);
    Vec tolo = make_vec(g, plo, 3, ncol, 1, 1, s);
    if (!to64.ok() || !tolo.ok()) return fail(LQ_ENOMEM, "HISQ buffers");
    OpFn A64 = [&](Vec& o, const Vec& i) {
      Vec t = view(to64, 0, i.ncol);
      return stag_normal_even(env, 64, o, i, t, dm2.as<double>(), 0.0);
    };
    OpFn Alo = [&](Vec& o, const Vec& i) {
      Vec t = view(tolo, 0, i.ncol);
      return stag_normal_even(env, plo, o, i, t, dm2.as<double>(), 0.0);
    };
    FusedFn Afused = [&](Vec& o, const Vec& i, int, double* red) {
      Vec t = view(tolo, 0, i.ncol);
      return stag_normal_even(env, plo, o, i, t, dm2.as<double>(), 0.0, red);
    };
    // target half the tolerance, so the result keeps a margin below it; a
    // column still above the tolerance (rounding in the last update) goes
    // round again from its iterate with a tighter target
    std::vector<double> tolv(ncol, 0.5 * tol);
    ColParam cpm{m2col, dm2.as<double>(), s};  // m^2 per column follows the solver's reordering
    std::vector<double> res;
    for (int pass = 0; pass < 4; ++pass) {
      const int rs = cg_mixed(ble, g, A64, Alo, plo, y, brep, tolv, maxiter, delta, cnt, &cpm, &Afused);
      if (rs != LQ_OK && rs != LQ_ENOCONV) return rs;
      status = rs;
      if ((e = rel_residual(ble, A64, y, brep, res, g))) return e;
      worst = *std::max_element(res.begin(), res.end());
      if (worst <= tol || rs == LQ_ENOCONV) break;
      for (int k = 0; k < ncol; ++k)
        if (res[k] > tol) tolv[k] *= std::max(0.05, 0.5 * tol / res[k]);
    }
    // output
    const size_t colsz = (size_t)2 * g.Vh * 3 * 2;  // doubles per column
    if (launch_fill_zero(x_dev, sizeof(double) * colsz * ncol, s)) return fail(LQ_EDEVICE, "zero");
    Vec yo;
    if (prm->reconstruct_full) {
      Vec yf = make_vec(g, 64, 3, ncol, 2, 0, s);
      yo = make_vec(g, 64, 3, ncol, 2, 0, s);
      if (!yf.ok() || !yo.ok()) return fail(LQ_ENOMEM, "reconstruct buffers");
      if ((e = vec_zero(yf))) return e;
      for (int k = 0; k < ncol; ++k) {
        FieldRef dst = yf.cols(k), src = y.cols(k);
        if (launch_convert(dst, 64, src, 64, 3, 1, 1, g.Vh, s)) return fail(LQ_EDEVICE, "copy");
      }
      if ((e = stag_D(env, 64, yo, yf, true, dm.as<double>()))) return e;
    }
    for (int k = 0; k < nsh; ++k) {
      double* dst = x_dev + (size_t)order[k] * n_rhs * colsz;
      if (prm->reconstruct_full) {
        Vec v = view(yo, k * n_rhs, n_rhs);
        if (launch_unpack_field(g, v.f, 64, n_rhs, 3, dst, 2, s)) return fail(LQ_EDEVICE, "unpack");
      } else {
        Vec v = view(y, k * n_rhs, n_rhs);
        if (launch_unpack_field(g, v.f, 64, n_rhs, 3, dst, 0, s)) return fail(LQ_EDEVICE, "unpack");
      }
    }
  } else {
    return fail(LQ_EINVAL, "unknown action kind");
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "solve synchronise");
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    stats->iters = cnt.iters;
    stats->reliable_updates = cnt.reliable;
    stats->true_rel_res = worst;
    stats->seconds = secs;
    stats->gflops = secs > 0 ? env.flops / secs * 1e-9 : 0;
    stats->hbm_bytes = env.bytes;
    stats->n_apply = (int32_t)std::min<int64_t>(env.n_apply, INT32_MAX);
    stats->status = status;
  }
  if (status == LQ_ENOCONV) return fail(LQ_ENOCONV, "maximum iterations reached before the target residual");
  return LQ_OK;
}

// ------------------------------------------------------------------ single application
int apply_op(lq_ctx* c, const lq_action* act, lq_field* f, int op, int prec, int n_rhs, const double* in_dev,
             double* out_dev, hipStream_t s) {
  const Geom& g = f->g;
  OpEnv env{c, f, *act, s};
  env.recon = (prec & LQ_PREC_RECON12) ? 1 : 0;
  prec &= ~LQ_PREC_RECON12;
  const int kind = act->kind;
  const int nc = kind == LQ_HISQ ? 3 : 12;
  if ((kind == LQ_HISQ) != (f->type == 1)) return fail(LQ_EINVAL, "field type does not match the action");
  Vec in = make_vec(g, prec, nc, n_rhs, 2, 0, s);
  Vec out = make_vec(g, prec, nc, n_rhs, 2, 0, s);
  if (!in.ok() || !out.ok()) return fail(LQ_ENOMEM, "apply buffers");
  if (launch_pack_field(g, in_dev, n_rhs, nc, in.f, prec, 2, s)) return fail(LQ_EDEVICE, "pack");
  int e = 0;
  int par_sel = 2;
  if (kind == LQ_HISQ) {
    if (op == LQ_OP_D) e = stag_D(env, prec, out, in, false);
    else if (op == LQ_OP_DDAG) e = stag_D(env, prec, out, in, true);
    else if (op == LQ_OP_HOP) e = stag_hop(env, prec, out, in);
    else if (op == LQ_OP_NORMAL_EVEN) {
      Vec ie = make_vec(g, prec, 3, n_rhs, 1, 0, s), oe = make_vec(g, prec, 3, n_rhs, 1, 0, s),
          to = make_vec(g, prec, 3, n_rhs, 1, 1, s);
      if (!ie.ok() || !oe.ok() || !to.ok()) return fail(LQ_ENOMEM, "apply buffers");
      if (launch_pack_field(g, in_dev, n_rhs, 3, ie.f, prec, 0, s)) return fail(LQ_EDEVICE, "pack");
      if ((e = stag_normal_even(env, prec, oe, ie, to, nullptr, act->m * act->m))) return e;
      if (launch_fill_zero(out_dev, sizeof(double) * 2 * 3 * 2 * (size_t)g.Vh * n_rhs, s)) return fail(LQ_EDEVICE, "zero");
      if (launch_unpack_field(g, oe.f, prec, n_rhs, 3, out_dev, 0, s)) return fail(LQ_EDEVICE, "unpack");
      return hipStreamSynchronize(s) == hipSuccess ? 0 : fail(LQ_EDEVICE, "sync");
    } else return fail(LQ_EINVAL, "op not defined for HISQ");
  } else {
    if (kind == LQ_OVERLAP && prec == 64 && op != LQ_OP_HW && op != LQ_OP_HOP) {
      if ((e = overlap_prepare(env))) return e;
    }
    switch (op) {
      case LQ_OP_D:
      case LQ_OP_DDAG:
        if (kind == LQ_OVERLAP) {
          if ((e = overlap_prepare(env))) return e;
          e = overlap_D(env, prec, out, in, op == LQ_OP_DDAG);
        } else {
          e = wilson_D(env, prec, out, in, op == LQ_OP_DDAG);
        }
        break;
      case LQ_OP_HOP: e = wilson_hop(env, prec, out, in); break;
      case LQ_OP_SITE:
      case LQ_OP_SITE_INV:
        if (kind != LQ_TM_CLOVER) return fail(LQ_EINVAL, "site term needs the twisted-clover action");
        e = tm_site(env, prec, out, in, op == LQ_OP_SITE_INV);
        break;
      case LQ_OP_SCHUR: {
        if (kind != LQ_TM_CLOVER) return fail(LQ_EINVAL, "Schur operator needs the twisted-clover action");
        Vec ie = make_vec(g, prec, 12, n_rhs, 1, 0, s), oe = make_vec(g, prec, 12, n_rhs, 1, 0, s),
            to = make_vec(g, prec, 12, n_rhs, 1, 1, s);
        if (!ie.ok() || !oe.ok() || !to.ok()) return fail(LQ_ENOMEM, "apply buffers");
        if (launch_pack_field(g, in_dev, n_rhs, 12, ie.f, prec, 0, s)) return fail(LQ_EDEVICE, "pack");
        if ((e = tm_schur(env, prec, oe, ie, to))) return e;
        if (launch_fill_zero(out_dev, sizeof(double) * 2 * 12 * 2 * (size_t)g.Vh * n_rhs, s))
          return fail(LQ_EDEVICE, "zero");
        if (launch_unpack_field(g, oe.f, prec, n_rhs, 12, out_dev, 0, s)) return fail(LQ_EDEVICE, "unpack");
        return hipStreamSynchronize(s) == hipSuccess ? 0 : fail(LQ_EDEVICE, "sync");
      }
      case LQ_OP_HW: e = hw_apply(env, prec, out, in); break;
      case LQ_OP_SIGN:
        if (kind != LQ_OVERLAP) return fail(LQ_EINVAL, "sign function needs the overlap action");
        if ((e = overlap_prepare(env))) return e;
        e = sign_apply(env, prec, out, in);
        break;
      default: return fail(LQ_EINVAL, "op not defined for this action");
    }
  }
  if (e) return e;
  if (launch_unpack_field(g, out.f, prec, n_rhs, nc, out_dev, par_sel, s)) return fail(LQ_EDEVICE, "unpack");
  return hipStreamSynchronize(s) == hipSuccess ? 0 : fail(LQ_EDEVICE, "sync");
}

int apply_op_noalloc(lq_ctx* c, const lq_action* act, lq_field* f, int op, int prec, int n_rhs,
                     const double* in_dev, double* out_dev, hipStream_t s, void* scratch, size_t scratch_bytes) {
  const Geom& g = f->g;
  OpEnv env{c, f, *act, s};
  env.noalloc = true;
  env.recon = (prec & LQ_PREC_RECON12) ? 1 : 0;
  prec &= ~LQ_PREC_RECON12;
  const int kind = act->kind;
  const int nc = kind == LQ_HISQ ? 3 : 12;
  if ((kind == LQ_HISQ) != (f->type == 1)) return fail(LQ_EINVAL, "field type does not match the action");
  const bool ok_op = op == LQ_OP_D || op == LQ_OP_DDAG || op == LQ_OP_HOP;
  if (kind == LQ_OVERLAP ? op != LQ_OP_HW && op != LQ_OP_HOP : !ok_op)
    return fail(LQ_EINVAL, "lq_apply_noalloc: op must be D, D^dag or the hopping term (H_W or the hopping term "
                           "for overlap)");
  if (!scratch) return fail(LQ_EDEVICE, "lq_apply_noalloc: scratch not set up on this device");
  const size_t vb = vec_bytes(g, prec, nc, n_rhs, 2);
  const size_t vbr = (vb + 255) / 256 * 256;
  if (2 * vbr > scratch_bytes)
    return fail(LQ_EINVAL, "lq_apply_noalloc: " + std::to_string(n_rhs) + " columns need " +
                               std::to_string(2 * vbr) + " bytes of scratch, the maximum is " +
                               std::to_string(scratch_bytes));
  Vec in = vec_at(g, prec, nc, n_rhs, 2, 0, scratch, s);
  Vec out = vec_at(g, prec, nc, n_rhs, 2, 0, (char*)scratch + vbr, s);
  if (launch_pack_field(g, in_dev, n_rhs, nc, in.f, prec, 2, s)) return fail(LQ_EDEVICE, "pack");
  int e = 0;
  if (kind == LQ_HISQ) {
    if (op == LQ_OP_HOP) e = stag_hop(env, prec, out, in);
    else e = stag_D(env, prec, out, in, op == LQ_OP_DDAG);
  } else if (op == LQ_OP_HOP) {
    e = wilson_hop(env, prec, out, in);
  } else if (op == LQ_OP_HW) {
    e = hw_apply(env, prec, out, in);
  } else {
    e = wilson_D(env, prec, out, in, op == LQ_OP_DDAG);
  }
  if (e) return e;
  if (launch_unpack_field(g, out.f, prec, n_rhs, nc, out_dev, 2, s)) return fail(LQ_EDEVICE, "unpack");
  return 0;
}

// ------------------------------------------------------------------ Lanczos bounds
static void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lo, double& hi) {
  // bisection with Sturm counts on the symmetric tridiagonal (a diagonal, b off-diagonal)
  const int n = (int)a.size();
  double gl = 1e300, gu = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i < n - 1 ? std::fabs(b[i]) : 0);
    gl = std::min(gl, a[i] - r);
    gu = std::max(gu, a[i] + r);
  }
  auto count = [&](double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int k) {
    double l = gl, u = gu;
    for (int it = 0; it < 200; ++it) {
      const double m = 0.5 * (l + u);
      if (count(m) > k) u = m;
      else l = m;
    }
    return 0.5 * (l + u);
  };
  lo = kth(0);
  hi = kth(n - 1);
}

// Solves (T - mu) y = y in place for the symmetric tridiagonal T (diagonal a,
// off-diagonal b) by Gaussian elimination with partial pivoting; the factor
// of a tridiagonal matrix then has two super-diagonals.
static void tri_shift_solve(const std::vector<double>& a, const std::vector<double>& b, double mu,
                            std::vector<double>& y) {
  const int n = (int)a.size();
  std::vector<double> d(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a[i] - mu;
  for (int i = 0; i + 1 < n; ++i) du[i] = dl[i] = b[i];
  std::vector<char> piv(n, 0);
  for (int i = 0; i + 1 < n; ++i) {
    if (std::fabs(d[i]) >= std::fabs(dl[i])) {
      const double f = d[i] != 0.0 ? dl[i] / d[i] : 0.0;
      dl[i] = f;
      d[i + 1] -= f * du[i];
    } else {
      // exchange rows i and i+1
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = d[i + 1];
      d[i + 1] = t - f * d[i + 1];
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
      piv[i] = 1;
    }
  }
  for (int i = 0; i < n; ++i)
    if (d[i] == 0.0) d[i] = 1e-300;
  for (int i = 0; i + 1 < n; ++i) {
    if (piv[i]) std::swap(y[i], y[i + 1]);
    y[i + 1] -= dl[i] * y[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = y[i];
    if (i + 1 < n) v -= du[i] * y[i + 1];
    if (i + 2 < n) v -= du2[i] * y[i + 2];
    y[i] = v / d[i];
  }
}

// unit eigenvector of T for the eigenvalue theta by inverse iteration
static std::vector<double> tri_eigvec(const std::vector<double>& a, const std::vector<double>& b, double theta) {
  const int n = (int)a.size();
  std::vector<double> y(n, 1.0 / std::sqrt((double)std::max(n, 1)));
  const double mu = theta + 1e-13 * std::max(1.0, std::fabs(theta));
  for (int it = 0; it < 4; ++it) {
    tri_shift_solve(a, b, mu, y);
    double nn = 0.0;
    for (double v : y) nn += v * v;
    nn = std::sqrt(nn);
    if (!(nn > 0) || !std::isfinite(nn)) break;
    for (double& v : y) v /= nn;
  }
  return y;
}

// Interval of the spectrum of H_W^2 (sec. 2.3: the Chebyshev interval must
// hold it).  FP64 Lanczos from a fixed random start vector gives the
// tridiagonal T; Sturm bisection gives its extreme eigenvalues theta_min and
// theta_max, inverse iteration their eigenvectors s.  A second Lanczos pass
// (deterministic reductions reproduce the same basis vectors v_j bit for bit)
// forms the Ritz vectors y = sum_j s_j v_j, and their residuals
// r = |H^2 y - theta y| / |y| are computed with the FP64 operator.  Some
// eigenvalue lies within r of each Ritz value, and Lanczos from a random
// start approaches the extreme eigenvalues from inside the spectrum, so
// [theta_min - r_min, theta_max + r_max] is taken to hold the spectrum.
// Lanczos counts as converged when r_min < theta_min / 2; otherwise LQ_EINVAL.
int hw_spectrum(lq_ctx* c, const lq_action* act, lq_field* f, int iters, HwSpectrum* out, hipStream_t s) {
  if (f->type != 0) return fail(LQ_EINVAL, "H_W bounds need a Wilson gauge field");
  if (iters < 2) return fail(LQ_EINVAL, "H_W bounds need at least 2 Lanczos steps");
  const Geom& g = f->g;
  OpEnv env{c, f, *act, s};
  Blas bl;
  int e = blas_prepare(c, bl, g, 2, 1, s);
  if (e) return e;
  const int64_t nd = 2 * (int64_t)g.Vh * 24;
  std::vector<double> h(nd);
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd01;
  for (auto& v : h) v = nd01(rng);
  DBuf raw(sizeof(double) * nd, s);
  Vec v = make_vec(g, 64, 12, 1, 2, 0, s), w = make_vec(g, 64, 12, 1, 2, 0, s),
      vp = make_vec(g, 64, 12, 1, 2, 0, s), t = make_vec(g, 64, 12, 1, 2, 0, s),
      ylo = make_vec(g, 64, 12, 1, 2, 0, s), yhi = make_vec(g, 64, 12, 1, 2, 0, s);
  if (!raw.p || !v.ok() || !w.ok() || !vp.ok() || !t.ok() || !ylo.ok() || !yhi.ok())
    return fail(LQ_ENOMEM, "lanczos buffers");
  hipMemcpyAsync(raw.p, h.data(), sizeof(double) * nd, hipMemcpyHostToDevice, s);
  State st(1, s);
  if (!st.ok()) return fail(LQ_ENOMEM, "lanczos state");
  std::vector<double> al, be;
  double beta_last = 0.0;
  // one Lanczos run; visit(j) sees the normalised basis vector v_j in v
  auto lanczos = [&](int m, const std::function<int(int)>& visit) -> int {
    int r = 0;
    al.clear();
    be.clear();
    if (launch_pack_field(g, raw.as<double>(), 1, 12, v.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
    std::vector<double> nn;
    if ((r = col_norms(bl, v, nn))) return r;
    if ((r = bl.opi(OP_SCALE, &v, nullptr, nullptr, 1.0 / std::sqrt(nn[0])))) return r;
    if ((r = vec_zero(vp))) return r;
    double beta_prev = 0.0;
    for (int j = 0; j < m; ++j) {
      if (visit && (r = visit(j))) return r;
      if ((r = hw_apply(env, 64, t, v)) || (r = hw_apply(env, 64, w, t))) return r;  // w = H^2 v
      if ((r = bl.op(OP_DOT, &v, &w))) return r;
      if (launch_scalar(SC_DOT_TO_AUX, bl.partial, bl.gridx, 1, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
      if ((r = st.pull())) return r;
      const double alpha = st.h(0, ST_AUX);
      al.push_back(alpha);
      // w = w - alpha v - beta_prev vp
      if ((r = bl.opi(OP_AXMY, &v, &w, nullptr, alpha))) return r;
      if ((r = bl.opi(OP_AXMY, &vp, &w, nullptr, beta_prev))) return r;
      if ((r = col_norms(bl, w, nn))) return r;
      const double beta = std::sqrt(nn[0]);
      beta_last = beta;
      if (!(beta > 1e-14 * std::fabs(alpha)) || j == m - 1) break;
      be.push_back(beta);
      std::swap(vp, v);
      if ((r = bl.opi(OP_SCALE, &w, nullptr, nullptr, 1.0 / beta))) return r;
      std::swap(v, w);
      beta_prev = beta;
    }
    return 0;
  };
  if ((e = lanczos(iters, nullptr))) return e;
  const int m = (int)al.size();
  be.resize(m > 0 ? m - 1 : 0);
  double lo = 0, hi = 0;
  tridiag_extremes(al, be, lo, hi);
  const std::vector<double> slo = tri_eigvec(al, be, lo), shi = tri_eigvec(al, be, hi);
  const std::vector<double> a_keep = al, b_keep = be;
  if ((e = vec_zero(ylo)) || (e = vec_zero(yhi))) return e;
  e = lanczos(m, [&](int j) -> int {
    int r = bl.opi(OP_AXPY, &v, &ylo, nullptr, slo[j]);
    return r ? r : bl.opi(OP_AXPY, &v, &yhi, nullptr, shi[j]);
  });
  if (e) return e;
  if (al != a_keep) return fail(LQ_EDEVICE, "lanczos: second pass did not reproduce the basis");
  // r = |H^2 y - theta y| / |y|
  auto ritz_res = [&](Vec& y, double theta, double& res) -> int {
    int r = 0;
    std::vector<double> ny, nq;
    if ((r = col_norms(bl, y, ny))) return r;
    if ((r = hw_apply(env, 64, t, y)) || (r = hw_apply(env, 64, w, t))) return r;
    if ((r = bl.opi(OP_AXMY, &y, &w, nullptr, theta))) return r;
    if ((r = col_norms(bl, w, nq))) return r;
    res = ny[0] > 0 ? std::sqrt(nq[0] / ny[0]) : 1e300;
    return 0;
  };
  double rlo = 0, rhi = 0;
  if ((e = ritz_res(ylo, lo, rlo)) || (e = ritz_res(yhi, hi, rhi))) return e;
  out->theta_min = lo;
  out->theta_max = hi;
  out->r_min = rlo;
  out->r_max = rhi;
  out->steps = m;
  if (!(rlo < 0.5 * lo) || !std::isfinite(rhi))
    return fail(LQ_EINVAL, "Lanczos on H_W^2 has not converged: Ritz residual " + std::to_string(rlo) +
                               " of the smallest Ritz value " + std::to_string(lo) + " after " + std::to_string(m) +
                               " steps");
  return 0;
}

int hw_bounds(lq_ctx* c, const lq_action* act, lq_field* f, int iters, double* lmin, double* lmax, hipStream_t s) {
  HwSpectrum sp{};
  int e = hw_spectrum(c, act, f, iters, &sp, s);
  if (e) return e;
  *lmin = std::sqrt(std::max(sp.theta_min - sp.r_min, 0.0));
  *lmax = std::sqrt(sp.theta_max + sp.r_max);
  return 0;
}

// ------------------------------------------------------------------ multigrid setup
int mg_setup(lq_ctx* c, const lq_action* act, lq_field* f, const lq_mg_params* mp, lq_stats* st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!mp) return fail(LQ_EINVAL, "multigrid parameters are NULL");
  if (f->type != 0) return fail(LQ_EINVAL, "multigrid needs a Wilson gauge field");
  if (act->kind != LQ_TM_CLOVER) return fail(LQ_EINVAL, "multigrid is implemented for the twisted-clover action");
  const Geom& g = f->g;
  const int nv = mp->n_vec > 0 ? mp->n_vec : 30;
  if (nv % 6 != 0 || nv > 30) return fail(LQ_EINVAL, "n_vec must be 6, 12, 18, 24 or 30");
  if (mp->nu_pre < 0 || mp->nu_pre > 16 || mp->nu_post < 0 || mp->nu_post > 16 || mp->reserved != 0)
    return fail(LQ_EINVAL, "nu_pre and nu_post must be in [0, 16], reserved 0");
  for (int mu = 0; mu < 4; ++mu) {
    const int b = mp->block[mu];
    if (b < 2 || g.L[mu] % b != 0 || (g.L[mu] / b) % 2 != 0)
      return fail(LQ_EINVAL, "block extents must be >= 2 and divide the lattice into an even number of aggregates");
  }
  OpEnv env{c, f, *act, s};
  Counters cnt;
  Vec w = make_vec(g, 64, 12, nv, 2, 0, s);
  if (!w.ok()) return fail(LQ_ENOMEM, "multigrid setup vectors");
  int e = 0;
  if (mp->null_vecs) {
    const size_t bytes = (size_t)nv * 2 * g.Vh * 24 * sizeof(double);
    DBuf aos(bytes, s);
    if (!aos.p) return fail(LQ_ENOMEM, "multigrid setup vectors");
    if (hipMemcpyAsync(aos.p, mp->null_vecs, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(LQ_EDEVICE, "copy");
    if (launch_pack_field(g, aos.as<double>(), nv, 12, w.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
  } else {
    if (launch_mg_random(w.f, nv, mp->seed, s)) return fail(LQ_EDEVICE, "multigrid random vectors");
    const int passes = mp->setup_passes > 0 ? mp->setup_passes : 2;
    const int maxiter = mp->setup_maxiter > 0 ? mp->setup_maxiter : 200;
    const double tol = mp->setup_tol > 0 ? mp->setup_tol : 1e-4;
    if ((e = mg_null_vectors(env, w, passes, maxiter, tol, cnt))) return e;
  }
  auto* h = new MgHier;
  h->kind = act->kind;
  h->m = act->m;
  h->mu = act->mu;
  h->csw = act->c_sw;
  h->coarse_tol = mp->coarse_tol > 0 ? mp->coarse_tol : 0.1;
  h->coarse_maxiter = mp->coarse_maxiter > 0 ? mp->coarse_maxiter : 100;
  h->nu_post = mp->nu_post > 0 ? mp->nu_post : 4;
  h->gcr_kmax = mp->gcr_kmax > 0 ? mp->gcr_kmax : 8;
  h->nu_pre = mp->nu_pre > 0 ? mp->nu_pre : 0;
  if ((e = mg_init_maps(*h, g, mp->block, nv)) || (e = mg_build(env, *h, w))) {
    mg_release(h);
    return e;
  }
  h->setup_iters = cnt.iters;
  h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  {
    std::lock_guard<std::mutex> lk(f->mtx);
    mg_release(f->mg);
    f->mg = h;
  }
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = h->setup_iters;
    st->n_apply = env.n_apply;
    st->seconds = h->setup_seconds;
    st->status = LQ_OK;
  }
  return 0;
}

}  // namespace lq
