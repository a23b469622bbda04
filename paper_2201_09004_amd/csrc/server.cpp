// Serving loop with continuous batching.
//
// Requests (n_rhs columns of one propagator, sec. 2.1 and 2.2: 12 spin-colour
// columns for Wilson-type actions, colour columns for staggered) arrive on
// any thread.  A worker thread keeps one solver engine per (gauge field,
// action, solver parameters): an engine owns device buffers for `cap`
// columns and advances every column it holds by one Krylov iteration per
// step.  Columns join an engine at iteration boundaries when it has free
// slots, and leave it as soon as their FP64 true residual meets the target
// (the last column is moved into the freed slot, so the batch stays dense).
// Engines of different keys run on their own HIP streams; a step enqueues
// all engines first and then completes them, so their kernels overlap on
// the device.  A new engine is created only if its HBM footprint fits the
// budget (idle engines are evicted first); requests that do not fit wait.
//
// Engines: twisted-clover even-odd BiCGStab (FP32/FP64 sloppy, FP64 reliable
// updates, reductions fused into the Schur stencil) and HISQ single-mass
// mixed-precision CG on M_e(m) = m^2 - D_eo D_oe (returns the even-site
// solution y, as lq_solve with reconstruct_full = 0).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "lq_internal.h"
#include "solver_util.h"

namespace lq {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  lq_action act{};
  lq_field* f = nullptr;
  lq_params prm{};
  int n_rhs = 0;
  const double* b = nullptr;
  double* x = nullptr;
  lq_stats* st = nullptr;
  Clock::time_point t_submit, t_done;
  int cols_left = 0;
  int status = LQ_OK;
  bool done = false;
  bool queued = false;
  double worst = 0.0;
  int iters = 0;
};

std::string engine_key(const Request& r) {
  char k[256];
  snprintf(k, sizeof(k), "%p|%d|%.17g|%.17g|%.17g|%.17g|%d|%d|%.17g", (void*)r.f, r.act.kind, r.act.m, r.act.mu,
           r.act.c_sw, r.prm.tol, r.prm.sloppy_bits, r.prm.recon12, r.prm.reliable_delta);
  return k;
}

struct ColMeta {
  Request* req = nullptr;
  int j = 0;          // column index within the request
  double bb = 0.0;    // |b_hat|^2 of the (preconditioned) system
  double maxrr = 0.0; // max residual^2 since the last reliable update
  double tol = 0.0;   // tolerance on the preconditioned system
  int iters = 0;
};

class Engine {
 public:
  Engine(lq_ctx* c, const Request& r, int cap_) : ctx(c), f(r.f), act(r.act), prm(r.prm), g(r.f->g), cap(cap_) {}
  virtual ~Engine() {
    stp.reset();  // frees on the stream, which must still exist
    if (s) {
      hipStreamSynchronize(s);
      hipStreamDestroy(s);
    }
  }
  virtual int init() = 0;
  virtual int admit(Request* r, int j0, int n) = 0;
  virtual int step_enqueue() = 0;
  // completes the step; appends finished requests' columns to `done`
  virtual int step_finish(std::vector<Request*>& done) = 0;

  lq_ctx* ctx;
  lq_field* f;
  lq_action act;
  lq_params prm;
  Geom g;
  int cap;
  int w = 0;
  hipStream_t s = nullptr;
  size_t footprint = 0;
  std::string key;
  Clock::time_point last_used = Clock::now();
  std::vector<ColMeta> cols;
  std::unique_ptr<State> stp;  // per-column scalars of the Krylov recurrence
  // iterations a column of this engine needs (running mean over finished
  // columns; a first guess until one finishes), for the scheduler
  double iters_per_col = 300.0;
  int64_t finished_cols = 0;
  void column_finished(int iters) {
    ++finished_cols;
    iters_per_col += (iters - iters_per_col) / (double)std::min<int64_t>(finished_cols, 32);
  }
  // device work of one iteration, in site-column units (a twisted-clover
  // iteration is two Schur operators, about twice a HISQ one per site)
  double iter_cost() const { return (double)g.Vh * std::max(w, 1) * (act.kind == LQ_HISQ ? 1.0 : 2.0); }
  // work left: remaining iterations of the columns held, at this engine's cost per column-iteration
  double remaining_work() const {
    double it = 0.0;
    for (int c = 0; c < w; ++c) it += std::max(1.0, iters_per_col - cols[c].iters);
    return it * (double)g.Vh * (act.kind == LQ_HISQ ? 1.0 : 2.0);
  }
  int plo = 32;
  double delta = 0.1;
  int maxiter = 10000;

 protected:
  int make_stream() {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(LQ_EDEVICE, "stream");
    stp = std::make_unique<State>(cap, s);
    return stp->ok() ? 0 : fail(LQ_ENOMEM, "engine state");
  }
  int alloc(Vec& v, int prec, int nc, int npar, int par0) {
    v = make_vec(g, prec, nc, cap, npar, par0, s);
    if (!v.ok()) return fail(LQ_ENOMEM, "engine buffers");
    footprint += v.bytes;
    return 0;
  }
  // copy column `from` onto column `to` of every listed vector and of the state
  int move_col(std::initializer_list<Vec*> vs, int from, int to) {
    for (Vec* v : vs)
      if (launch_convert(v->cols(to), v->prec, v->cols(from), v->prec, v->nc, 1, v->npar, g.Vh, s))
        return fail(LQ_EDEVICE, "column move");
    for (int k = 0; k < ST_STRIDE; ++k) stp->h(to, k) = stp->h(from, k);
    cols[to] = cols[from];
    return 0;
  }
  // host column `j` of a request's field (doubles per column)
  size_t col_doubles(int nc) const { return (size_t)2 * g.Vh * nc * 2; }
};

// ---------------------------------------------------------------- twisted clover
class TmEngine : public Engine {
 public:
  using Engine::Engine;
  int init() override {
    plo = prm.sloppy_bits == 64 ? 64 : 32;
    if (make_stream()) return LQ_EDEVICE;
    env = std::make_unique<OpEnv>(OpEnv{ctx, f, act, s});
    env->recon = prm.recon12;
    int e = 0;
    if ((e = alloc(bfull, 64, 12, 2, 0)) || (e = alloc(bhat, 64, 12, 1, 0)) || (e = alloc(xe, 64, 12, 1, 0)) ||
        (e = alloc(r64, 64, 12, 1, 0)) || (e = alloc(to64, 64, 12, 1, 1)) || (e = alloc(rs, plo, 12, 1, 0)) ||
        (e = alloc(rhat, plo, 12, 1, 0)) || (e = alloc(p, plo, 12, 1, 0)) || (e = alloc(v, plo, 12, 1, 0)) ||
        (e = alloc(t, plo, 12, 1, 0)) || (e = alloc(xs, plo, 12, 1, 0)) || (e = alloc(tolo, plo, 12, 1, 1)))
      return e;
    tiles = (g.Vh + 63) / 64;
    red = DBuf(sizeof(double) * 4 * (size_t)tiles * cap, s);
    stage = DBuf(sizeof(double) * col_doubles(12), s);
    if (!red.p || !stage.p) return fail(LQ_ENOMEM, "engine buffers");
    footprint += red.n + stage.n;
    if ((e = blas_prepare(ctx, ble, g, 1, cap, s)) || (e = blas_prepare(ctx, blf, g, 2, 1, s))) return e;
    if ((e = ensure_links(*env, plo)) || (e = ensure_links(*env, 64)) || (e = ensure_clover(*env, plo)) ||
        (e = ensure_clover(*env, 64)))
      return e;
    return 0;
  }

  static size_t estimate(const Geom& g, int cap, int plo) {
    const size_t blk64 = (size_t)g.Vh * 192, blklo = (size_t)g.Vh * (plo == 64 ? 192 : 96);
    return (size_t)cap * (6 * blk64 + 7 * blklo) + (size_t)g.Vh * 2 * 192;
  }

  int admit(Request* rq, int j0, int n) override {
    State& st = *stp;
    const int c0 = w;
    int e = 0;
    Vec bf = view(bfull, c0, n), bh = view(bhat, c0, n), xv = view(xe, c0, n), rv = view(rs, c0, n),
        rh = view(rhat, c0, n), pv = view(p, c0, n), xsv = view(xs, c0, n);
    // host b columns -> device -> even-odd layout
    DBuf raw(sizeof(double) * col_doubles(12) * n, s);
    if (!raw.p) return fail(LQ_ENOMEM, "admit staging");
    if (hipMemcpyAsync(raw.p, rq->b + (size_t)j0 * col_doubles(12), raw.n, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(LQ_EDEVICE, "upload");
    if (launch_pack_field(g, raw.as<double>(), n, 12, bf.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
    if ((e = tm_schur_source(*env, bh, bf))) return e;
    if ((e = vec_zero(xv)) || (e = vec_copy(rv, bh)) || (e = vec_copy(rh, rv)) || (e = vec_copy(pv, rv)) ||
        (e = vec_zero(xsv)))
      return e;
    std::vector<double> bb;
    Blas bln;
    if ((e = blas_prepare(ctx, bln, g, 1, n, s)) || (e = col_norms(bln, bh, bb))) return e;
    if ((e = bln.op(OP_DOT_NORM, &rv, &rh))) return e;
    if (launch_scalar(SC_SET_RHO_RR, bln.partial, bln.gridx, n, st.d() + (size_t)c0 * ST_STRIDE, s))
      return fail(LQ_EDEVICE, "scalar");
    for (int k = 0; k < n; ++k) {
      ColMeta m;
      m.req = rq;
      m.j = j0 + k;
      m.bb = bb[k];
      m.tol = 0.5 * (rq->prm.tol > 0 ? rq->prm.tol : 1e-10);
      cols.resize(std::max<size_t>(cols.size(), (size_t)c0 + k + 1));
      cols[c0 + k] = m;
    }
    // state rows of the new columns: keep rho, rr computed above; clear the rest
    if ((e = st.pull(c0 + n))) return e;
    for (int k = 0; k < n; ++k) {
      const double rho_re = st.h(c0 + k, ST_RHO), rho_im = st.h(c0 + k, ST_RHO + 1), rr = st.h(c0 + k, ST_RR);
      for (int q = 0; q < ST_STRIDE; ++q) st.h(c0 + k, q) = 0.0;
      st.h(c0 + k, ST_RHO) = rho_re;
      st.h(c0 + k, ST_RHO + 1) = rho_im;
      st.h(c0 + k, ST_RR) = rr;
      st.h(c0 + k, ST_ACTIVE) = 1.0;
      cols[c0 + k].maxrr = rr;
    }
    if ((e = st.push(c0 + n))) return e;
    w += n;
    return 0;
  }

  int step_enqueue() override {
    if (w == 0) return 0;
    State& st = *stp;
    Vec pv = view(p, 0, w), vv = view(v, 0, w), rv = view(rs, 0, w), tv = view(t, 0, w), xsv = view(xs, 0, w),
        rh = view(rhat, 0, w);
    Vec tov = view(tolo, 0, w);
    int e = 0;
    double* rb = red.as<double>();
    if ((e = tm_schur(*env, plo, vv, pv, tov))) return e;
    if ((e = ble.op(OP_DOT, &rh, &vv))) return e;
    if (launch_scalar(SC_BICG_ALPHA, ble.partial, ble.gridx, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if ((e = ble.op(OP_AXMY, &vv, &rv, nullptr, nullptr, nullptr, st.d(), ST_ALPHA, ST_ALPHA))) return e;
    if ((e = tm_schur(*env, plo, tv, rv, tov, 2, rb))) return e;
    if (launch_scalar(SC_BICG_OMEGA, rb, tiles, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if ((e = ble.op(OP_BICG_XR, &pv, &rv, &tv, &xsv, &rh, st.d(), ST_ALPHA, ST_OMEGA))) return e;
    if (launch_scalar(SC_BICG_BETA, ble.partial, ble.gridx, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if (hipMemcpyAsync(st.host.p, st.dev.p, (size_t)w * ST_STRIDE * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(LQ_EDEVICE, "state readback");
    return 0;
  }

  int step_finish(std::vector<Request*>& done) override {
    if (w == 0) return 0;
    State& st = *stp;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "engine step");
    last_used = Clock::now();
    bool breakdown = false;
    UpdateRule rule;
    for (int c = 0; c < w; ++c) {
      ColMeta& m = cols[c];
      ++m.iters;
      if (st.h(c, ST_FLAG) == 2.0 || !std::isfinite(st.h(c, ST_RR))) return fail(LQ_ENUMERIC, "NaN/Inf residual");
      if (st.h(c, ST_FLAG) == 1.0) breakdown = true;
      const double rr = st.h(c, ST_RR);
      m.maxrr = std::max(m.maxrr, rr);
      rule.column(rr, m.maxrr, m.tol * m.tol * m.bb, delta);
      if (m.iters >= maxiter) rule.now = true;
    }
    const bool update = rule.fire();
    Vec pv = view(p, 0, w), vv = view(v, 0, w), rv = view(rs, 0, w), xsv = view(xs, 0, w), rh = view(rhat, 0, w),
        xv = view(xe, 0, w), rr64 = view(r64, 0, w), bh = view(bhat, 0, w), to = view(to64, 0, w);
    int e = 0;
    std::vector<int> finished;
    if (update || breakdown) {
      // reliable update for every column: x += xs; r = b_hat - M x (FP64)
      if (launch_axpy_mixed(xv.f, 64, xsv.f, plo, 12, w, 1, g.Vh, s)) return fail(LQ_EDEVICE, "axpy");
      if ((e = vec_zero(xsv))) return e;
      if ((e = tm_schur(*env, 64, rr64, xv, to))) return e;
      if ((e = ble.op(OP_XMY_NORM, &bh, &rr64))) return e;
      if ((e = vec_copy(rv, rr64))) return e;
      if (breakdown) {
        if ((e = vec_copy(rh, rv)) || (e = vec_copy(pv, rv))) return e;
        for (int c = 0; c < w; ++c) st.h(c, ST_FLAG) = 0.0;
        if ((e = st.push(w))) return e;
      }
      if ((e = ble.op(OP_DOT_NORM, &rv, &rh))) return e;
      if (launch_scalar(SC_SET_RHO_RR, ble.partial, ble.gridx, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
      if ((e = st.pull(w))) return e;
      for (int c = 0; c < w; ++c) {
        ColMeta& m = cols[c];
        m.maxrr = st.h(c, ST_RR);
        if (st.h(c, ST_RR) <= m.tol * m.tol * m.bb || m.iters >= maxiter) finished.push_back(c);
      }
    }
    if (!breakdown) {
      if ((e = ble.op(OP_BICG_P, &rv, &vv, &pv, nullptr, nullptr, st.d(), ST_BETA, ST_OMEGA))) return e;
    }
    // retire finished columns, highest slot first so compaction keeps lower slots valid
    std::sort(finished.rbegin(), finished.rend());
    for (int c : finished) {
      ColMeta m = cols[c];
      double res = 0.0;
      if ((e = reconstruct_and_check(c, res))) return e;
      const double tol = m.req->prm.tol > 0 ? m.req->prm.tol : 1e-10;
      if (res > tol && m.iters < maxiter) {
        cols[c].tol *= std::max(0.05, 0.5 * tol / res);  // tighten and keep iterating
        continue;
      }
      if ((e = copy_out(c))) return e;
      Request* rq = m.req;
      rq->worst = std::max(rq->worst, res);
      rq->iters = std::max(rq->iters, m.iters);
      column_finished(m.iters);
      if (res > tol) rq->status = LQ_ENOCONV;
      if (--rq->cols_left == 0) done.push_back(rq);
      const int last = w - 1;
      if (c != last && (e = move_col({&bfull, &bhat, &xe, &rs, &rhat, &p, &xs}, last, c))) return e;
      --w;
    }
    if (!finished.empty() && w > 0 && (e = st.push(w))) return e;
    return 0;
  }

 private:
  // full solution of column c into `xfull` and its FP64 relative residual
  int reconstruct_and_check(int c, double& res) {
    int e = 0;
    Vec xf = make_vec(g, 64, 12, 1, 2, 0, s);
    if (!xf.ok()) return fail(LQ_ENOMEM, "reconstruct buffer");
    Vec xv = view(xe, c, 1), bf = view(bfull, c, 1);
    if ((e = tm_schur_reconstruct(*env, xf, xv, bf))) return e;
    OpFn D64 = [&](Vec& o, const Vec& i) { return wilson_D(*env, 64, o, i, false); };
    std::vector<double> r;
    if ((e = rel_residual(blf, D64, xf, bf, r, g))) return e;
    res = r[0];
    if (launch_unpack_field(g, xf.f, 64, 1, 12, stage.as<double>(), 2, s)) return fail(LQ_EDEVICE, "unpack");
    return 0;
  }
  int copy_out(int c) {
    const ColMeta& m = cols[c];
    if (hipMemcpyAsync(m.req->x + (size_t)m.j * col_doubles(12), stage.p, sizeof(double) * col_doubles(12),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LQ_EDEVICE, "download");
    return 0;
  }

  std::unique_ptr<OpEnv> env;
  Vec bfull, bhat, xe, r64, to64, rs, rhat, p, v, t, xs, tolo;
  DBuf red, stage;
  Blas ble, blf;
  int tiles = 1;
};

// ---------------------------------------------------------------- HISQ single mass
class HisqEngine : public Engine {
 public:
  using Engine::Engine;
  int init() override {
    plo = prm.sloppy_bits == 64 ? 64 : prm.sloppy_bits == 16 ? 16 : 32;
    if (make_stream()) return LQ_EDEVICE;
    env = std::make_unique<OpEnv>(OpEnv{ctx, f, act, s});
    int e = 0;
    if ((e = alloc(be, 64, 3, 1, 0)) || (e = alloc(y, 64, 3, 1, 0)) || (e = alloc(r64, 64, 3, 1, 0)) ||
        (e = alloc(to64, 64, 3, 1, 1)) || (e = alloc(rs, plo, 3, 1, 0)) || (e = alloc(p, plo, 3, 1, 0)) ||
        (e = alloc(q, plo, 3, 1, 0)) || (e = alloc(xs, plo, 3, 1, 0)) || (e = alloc(tolo, plo, 3, 1, 1)))
      return e;
    stage = DBuf(sizeof(double) * col_doubles(3), s);
    if (!stage.p) return fail(LQ_ENOMEM, "engine buffers");
    footprint += stage.n;
    if ((e = blas_prepare(ctx, ble, g, 1, cap, s))) return e;
    if ((e = ensure_links(*env, plo)) || (e = ensure_links(*env, 64))) return e;
    m2 = act.m * act.m;
    return 0;
  }

  static size_t estimate(const Geom& g, int cap, int plo) {
    const size_t blk64 = (size_t)g.Vh * 48, blklo = (size_t)g.Vh * (plo == 64 ? 48 : plo == 32 ? 24 : 16);
    return (size_t)cap * (4 * blk64 + 5 * blklo) + (size_t)g.Vh * 2 * 48;
  }

  int admit(Request* rq, int j0, int n) override {
    State& st = *stp;
    const int c0 = w;
    int e = 0;
    Vec bv = view(be, c0, n), yv = view(y, c0, n), rv = view(rs, c0, n), pv = view(p, c0, n), xsv = view(xs, c0, n);
    DBuf raw(sizeof(double) * col_doubles(3) * n, s);
    if (!raw.p) return fail(LQ_ENOMEM, "admit staging");
    if (hipMemcpyAsync(raw.p, rq->b + (size_t)j0 * col_doubles(3), raw.n, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(LQ_EDEVICE, "upload");
    if (launch_pack_field(g, raw.as<double>(), n, 3, bv.f, 64, 0, s)) return fail(LQ_EDEVICE, "pack");
    if ((e = vec_zero(yv)) || (e = vec_copy(rv, bv)) || (e = vec_copy(pv, rv)) || (e = vec_zero(xsv))) return e;
    std::vector<double> bb;
    Blas bln;
    if ((e = blas_prepare(ctx, bln, g, 1, n, s)) || (e = col_norms(bln, bv, bb))) return e;
    if ((e = st.pull(std::max(c0, 1)))) return e;
    for (int k = 0; k < n; ++k) {
      for (int qq = 0; qq < ST_STRIDE; ++qq) st.h(c0 + k, qq) = 0.0;
      st.h(c0 + k, ST_RR) = bb[k];
      st.h(c0 + k, ST_ACTIVE) = 1.0;
      ColMeta m;
      m.req = rq;
      m.j = j0 + k;
      m.bb = bb[k];
      m.maxrr = bb[k];
      m.tol = rq->prm.tol > 0 ? rq->prm.tol : 1e-10;
      cols.resize(std::max<size_t>(cols.size(), (size_t)c0 + k + 1));
      cols[c0 + k] = m;
    }
    if ((e = st.push(c0 + n))) return e;
    w += n;
    return 0;
  }

  int step_enqueue() override {
    if (w == 0) return 0;
    State& st = *stp;
    Vec pv = view(p, 0, w), qv = view(q, 0, w), rv = view(rs, 0, w), xsv = view(xs, 0, w), tov = view(tolo, 0, w);
    int e = 0;
    if ((e = stag_normal_even(*env, plo, qv, pv, tov, nullptr, m2))) return e;
    if ((e = ble.op(OP_DOT, &pv, &qv))) return e;
    if (launch_scalar(SC_CG_ALPHA, ble.partial, ble.gridx, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if ((e = ble.op(OP_CG, &pv, &qv, &xsv, &rv, nullptr, st.d(), ST_ALPHA, ST_ALPHA))) return e;
    if (launch_scalar(SC_CG_BETA, ble.partial, ble.gridx, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
    if (hipMemcpyAsync(st.host.p, st.dev.p, (size_t)w * ST_STRIDE * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(LQ_EDEVICE, "state readback");
    return 0;
  }

  int step_finish(std::vector<Request*>& done) override {
    if (w == 0) return 0;
    State& st = *stp;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(LQ_EDEVICE, "engine step");
    last_used = Clock::now();
    UpdateRule rule;
    // (a column that lost positivity of <p, A p> took no step; SC_CG_BETA
    // restarted its direction on the device)
    for (int c = 0; c < w; ++c) {
      ColMeta& m = cols[c];
      ++m.iters;
      if (st.h(c, ST_FLAG) == 2.0 || !std::isfinite(st.h(c, ST_RR))) return fail(LQ_ENUMERIC, "NaN/Inf residual");
      const double rr = st.h(c, ST_RR);
      m.maxrr = std::max(m.maxrr, rr);
      rule.column(rr, m.maxrr, m.tol * m.tol * m.bb, delta);
      if (m.iters >= maxiter) rule.now = true;
    }
    const bool update = rule.fire();
    Vec pv = view(p, 0, w), rv = view(rs, 0, w), xsv = view(xs, 0, w), yv = view(y, 0, w), bv = view(be, 0, w),
        rr64 = view(r64, 0, w), to = view(to64, 0, w);
    int e = 0;
    std::vector<int> finished;
    if (update) {
      if (launch_axpy_mixed(yv.f, 64, xsv.f, plo, 3, w, 1, g.Vh, s)) return fail(LQ_EDEVICE, "axpy");
      if ((e = vec_zero(xsv))) return e;
      if ((e = stag_normal_even(*env, 64, rr64, yv, to, nullptr, m2))) return e;
      if ((e = ble.op(OP_XMY_NORM, &bv, &rr64))) return e;
      if (launch_scalar(SC_SET_RR, ble.partial, ble.gridx, w, st.d(), s)) return fail(LQ_EDEVICE, "scalar");
      if ((e = vec_copy(rv, rr64))) return e;
      if ((e = st.pull(w))) return e;
      for (int c = 0; c < w; ++c) {
        ColMeta& m = cols[c];
        m.maxrr = st.h(c, ST_RR);
        if (st.h(c, ST_RR) <= m.tol * m.tol * m.bb || m.iters >= maxiter) finished.push_back(c);
      }
    }
    if ((e = ble.op(OP_XPAY, &rv, &pv, nullptr, nullptr, nullptr, st.d(), ST_BETA, ST_BETA))) return e;
    std::sort(finished.rbegin(), finished.rend());
    for (int c : finished) {
      ColMeta m = cols[c];
      const double res = m.bb > 0 ? std::sqrt(st.h(c, ST_RR) / m.bb) : 0.0;
      Vec yc = view(y, c, 1);
      if (launch_fill_zero(stage.p, stage.n, s) ||
          launch_unpack_field(g, yc.f, 64, 1, 3, stage.as<double>(), 0, s))
        return fail(LQ_EDEVICE, "unpack");
      if (hipMemcpyAsync(m.req->x + (size_t)m.j * col_doubles(3), stage.p, stage.n, hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(LQ_EDEVICE, "download");
      Request* rq = m.req;
      rq->worst = std::max(rq->worst, res);
      rq->iters = std::max(rq->iters, m.iters);
      column_finished(m.iters);
      if (res > m.tol) rq->status = LQ_ENOCONV;
      if (--rq->cols_left == 0) done.push_back(rq);
      const int last = w - 1;
      if (c != last && (e = move_col({&be, &y, &rs, &p, &xs}, last, c))) return e;
      --w;
    }
    if (!finished.empty() && w > 0 && (e = st.push(w))) return e;
    return 0;
  }

 private:
  std::unique_ptr<OpEnv> env;
  Vec be, y, r64, to64, rs, p, q, xs, tolo;
  DBuf stage;
  Blas ble;
  double m2 = 0.0;
};

}  // namespace

struct ServerImpl {
  lq_ctx* ctx = nullptr;
  size_t budget = 0;
  int max_cols = 12;
  std::mutex m;
  std::condition_variable cv, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::unique_ptr<Engine>> engines;
  size_t used = 0;
  std::thread worker;
  bool stop = false;
  uint64_t next_id = 1;
  std::vector<double> latencies;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  int64_t cols_done = 0;
};

}  // namespace lq

struct lq_server {
  lq::ServerImpl impl;
};

namespace lq {
namespace {

void finish_request(ServerImpl& S, Request* rq, int status) {
  rq->t_done = Clock::now();
  if (status != LQ_OK && rq->status == LQ_OK) rq->status = status;
  if (rq->st) {
    rq->st->iters = rq->iters;
    rq->st->true_rel_res = rq->worst;
    rq->st->seconds = std::chrono::duration<double>(rq->t_done - rq->t_submit).count();
    rq->st->status = rq->status;
  }
  rq->done = true;
  S.latencies.push_back(std::chrono::duration<double>(rq->t_done - rq->t_submit).count());
  S.cols_done += rq->n_rhs;
  S.t_last = rq->t_done;
}

Engine* engine_for(ServerImpl& S, Request* rq, int& status) {
  const std::string key = engine_key(*rq);
  for (auto& e : S.engines)
    if (e->key == key) return e.get();
  const int plo = rq->prm.sloppy_bits == 64 ? 64 : rq->prm.sloppy_bits == 16 ? 16 : 32;
  const size_t need = rq->act.kind == LQ_HISQ ? HisqEngine::estimate(rq->f->g, S.max_cols, plo)
                                              : TmEngine::estimate(rq->f->g, S.max_cols, plo);
  if (need > S.budget) {
    status = fail(LQ_ENOMEM, "the engine for this request does not fit the server's HBM budget");
    return nullptr;
  }
  // evict idle engines, least recently used first, until the new one fits
  while (S.used + need > S.budget) {
    int victim = -1;
    for (int i = 0; i < (int)S.engines.size(); ++i)
      if (S.engines[i]->w == 0 && (victim < 0 || S.engines[i]->last_used < S.engines[victim]->last_used)) victim = i;
    if (victim < 0) return nullptr;  // wait for running columns to finish
    S.used -= S.engines[victim]->footprint;
    S.engines.erase(S.engines.begin() + victim);
  }
  std::unique_ptr<Engine> e;
  if (rq->act.kind == LQ_HISQ) e = std::make_unique<HisqEngine>(S.ctx, *rq, S.max_cols);
  else e = std::make_unique<TmEngine>(S.ctx, *rq, S.max_cols);
  e->key = key;
  e->delta = rq->prm.reliable_delta > 0 ? rq->prm.reliable_delta : 0.1;
  e->maxiter = rq->prm.maxiter > 0 ? rq->prm.maxiter : 10000;
  const int r = e->init();
  if (r) {
    status = r;
    return nullptr;
  }
  S.used += e->footprint;
  S.engines.push_back(std::move(e));
  return S.engines.back().get();
}

void worker_loop(ServerImpl& S) {
  hipSetDevice(S.ctx->device);
  for (;;) {
    std::vector<Request*> admit_now;
    {
      std::unique_lock<std::mutex> lk(S.m);
      auto busy = [&] {
        for (auto& e : S.engines)
          if (e->w > 0) return true;
        return false;
      };
      S.cv.wait(lk, [&] { return S.stop || !S.pending.empty() || busy(); });
      if (S.stop && S.pending.empty() && !busy()) return;
      admit_now.assign(S.pending.begin(), S.pending.end());
    }
    // admission at the iteration boundary, in arrival order; a request that does not fit yet
    // waits without holding back later requests that do
    std::vector<Request*> admitted;
    for (Request* rq : admit_now) {
      int status = LQ_OK;
      Engine* e = engine_for(S, rq, status);
      if (!e) {
        if (status != LQ_OK) {
          std::lock_guard<std::mutex> lk(S.m);
          finish_request(S, rq, status);
          admitted.push_back(rq);
          S.cv_done.notify_all();
        }
        continue;
      }
      if (e->w + rq->n_rhs > e->cap) continue;
      const int r = e->admit(rq, 0, rq->n_rhs);
      if (r) {
        std::lock_guard<std::mutex> lk(S.m);
        finish_request(S, rq, r);
        S.cv_done.notify_all();
      }
      admitted.push_back(rq);
    }
    if (!admitted.empty()) {
      std::lock_guard<std::mutex> lk(S.m);
      for (Request* rq : admitted) {
        auto it = std::find(S.pending.begin(), S.pending.end(), rq);
        if (it != S.pending.end()) S.pending.erase(it);
        rq->queued = false;
      }
    }
    // One cycle: every engine with columns advances one iteration (all are
    // enqueued first, so their kernels overlap on the device).  The engine
    // with the least remaining work advances more iterations while the
    // others' are in flight, about as many as fit in the costliest engine's
    // iteration (at most 8): short requests finish in proportion to their
    // own work instead of waiting one cycle of every engine per iteration.
    std::vector<Engine*> failed;
    Engine* first = nullptr;
    double cost_max = 0.0;
    for (auto& e : S.engines) {
      if (e->w == 0) continue;
      cost_max = std::max(cost_max, e->iter_cost());
      if (!first || e->remaining_work() < first->remaining_work()) first = e.get();
    }
    for (auto& e : S.engines)
      if (e->w > 0 && e->step_enqueue()) failed.push_back(e.get());
    std::vector<Request*> done;
    auto is_failed = [&](Engine* e) { return std::find(failed.begin(), failed.end(), e) != failed.end(); };
    if (first && !is_failed(first)) {
      int extra = std::min(8, (int)std::floor(cost_max / first->iter_cost())) - 1;
      if (first->step_finish(done)) failed.push_back(first);
      for (; extra > 0 && first->w > 0 && !is_failed(first); --extra)
        if (first->step_enqueue() || first->step_finish(done)) failed.push_back(first);
    }
    for (auto& e : S.engines) {
      if (e.get() == first || e->w == 0 || is_failed(e.get())) continue;
      if (e->step_finish(done)) failed.push_back(e.get());
    }
    {
      std::lock_guard<std::mutex> lk(S.m);
      for (Request* rq : done) finish_request(S, rq, LQ_OK);
      for (Engine* e : failed) {
        // fail every request that has a column in this engine, then drop the engine
        for (int c = 0; c < e->w; ++c) {
          Request* rq = e->cols[c].req;
          if (!rq->done) finish_request(S, rq, LQ_EDEVICE);
        }
        S.used -= e->footprint;
        S.engines.erase(std::find_if(S.engines.begin(), S.engines.end(),
                                     [&](const std::unique_ptr<Engine>& p) { return p.get() == e; }));
      }
      if (!done.empty() || !failed.empty()) S.cv_done.notify_all();
    }
  }
}

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" {

lq_status lq_server_create(lq_ctx* c, size_t hbm_budget, int max_cols, lq_server** srv) {
  if (!c || !srv) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  if (max_cols < 1 || max_cols > 256) return (lq_status)fail(LQ_EINVAL, "max_cols must be in [1, 256]");
  auto* s = new lq_server();
  s->impl.ctx = c;
  s->impl.budget = hbm_budget;
  s->impl.max_cols = max_cols;
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    hipSetDevice(c->device);
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) s->impl.budget = fr / 10 * 8;
  }
  s->impl.worker = std::thread([s] { worker_loop(s->impl); });
  *srv = s;
  return LQ_OK;
}

lq_status lq_server_destroy(lq_server* srv) {
  if (!srv) return (lq_status)fail(LQ_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(srv->impl.m);
    srv->impl.stop = true;
  }
  srv->impl.cv.notify_all();
  if (srv->impl.worker.joinable()) srv->impl.worker.join();
  srv->impl.engines.clear();
  delete srv;
  return LQ_OK;
}

lq_status lq_submit(lq_server* srv, const lq_action* act, const lq_field* g, const lq_params* prm, int n_rhs,
                    const double* b, double* x, lq_stats* st, uint64_t* ticket) {
  if (!srv || !act || !g || !prm || !b || !x || !ticket) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  if (act->kind != LQ_TM_CLOVER && act->kind != LQ_HISQ)
    return (lq_status)fail(LQ_ENOTSUP, "the server batches twisted-clover and HISQ solves");
  if ((act->kind == LQ_HISQ) != (g->type == 1)) return (lq_status)fail(LQ_EINVAL, "field type does not match");
  if (act->kind == LQ_HISQ && (prm->n_shift > 1 || !(act->m > 0)))
    return (lq_status)fail(LQ_EINVAL, "the server solves one positive HISQ mass per request");
  if (act->kind == LQ_TM_CLOVER && prm->sloppy_bits == 16)
    return (lq_status)fail(LQ_ENOTSUP, "twisted-clover sloppy storage is FP32 or FP64");
  if (n_rhs < 1 || n_rhs > srv->impl.max_cols) return (lq_status)fail(LQ_EINVAL, "n_rhs must be in [1, max_cols]");
  auto rq = std::make_unique<Request>();
  rq->act = *act;
  rq->f = const_cast<lq_field*>(g);
  rq->prm = *prm;
  rq->n_rhs = n_rhs;
  rq->b = b;
  rq->x = x;
  rq->st = st;
  rq->cols_left = n_rhs;
  rq->t_submit = Clock::now();
  rq->queued = true;
  if (st) std::memset(st, 0, sizeof(*st));
  {
    std::lock_guard<std::mutex> lk(srv->impl.m);
    rq->id = srv->impl.next_id++;
    *ticket = rq->id;
    if (!srv->impl.have_first) {
      srv->impl.have_first = true;
      srv->impl.t_first = rq->t_submit;
    }
    srv->impl.pending.push_back(rq.get());
    srv->impl.reqs[rq->id] = std::move(rq);
  }
  srv->impl.cv.notify_all();
  return LQ_OK;
}

lq_status lq_poll(lq_server* srv, uint64_t ticket, int* done) {
  if (!srv || !done) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->impl.m);
  auto it = srv->impl.reqs.find(ticket);
  if (it == srv->impl.reqs.end()) return (lq_status)fail(LQ_EINVAL, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return LQ_OK;
}

lq_status lq_wait(lq_server* srv, uint64_t ticket) {
  if (!srv) return (lq_status)fail(LQ_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->impl.m);
  auto it = srv->impl.reqs.find(ticket);
  if (it == srv->impl.reqs.end()) return (lq_status)fail(LQ_EINVAL, "unknown ticket");
  Request* rq = it->second.get();
  srv->impl.cv_done.wait(lk, [&] { return rq->done; });
  const int st = rq->status;
  if (st != LQ_OK) return (lq_status)fail(st, "request finished with an error status");
  return LQ_OK;
}

lq_status lq_server_stats(lq_server* srv, double* p50, double* p99, double* sps) {
  if (!srv || !p50 || !p99 || !sps) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->impl.m);
  std::vector<double> l = srv->impl.latencies;
  if (l.empty()) {
    *p50 = *p99 = *sps = 0.0;
    return LQ_OK;
  }
  std::sort(l.begin(), l.end());
  auto q = [&](double f) {
    const double pos = f * (l.size() - 1);
    const size_t i = (size_t)pos;
    const double fr = pos - i;
    return i + 1 < l.size() ? l[i] * (1 - fr) + l[i + 1] * fr : l[i];
  };
  *p50 = q(0.50);
  *p99 = q(0.99);
  const double span = std::chrono::duration<double>(srv->impl.t_last - srv->impl.t_first).count();
  *sps = span > 0 ? srv->impl.cols_done / span : 0.0;
  return LQ_OK;
}

}  // extern "C"
