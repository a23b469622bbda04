// extern "C" entry points of liblq (declared in include/lq.h): argument
// validation, host <-> device staging, and dispatch to the operators and
// solvers.  No entry point aborts; errors return a negative lq_status and set
// the thread-local message read by lq_last_error().
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "lq_internal.h"

namespace lq {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

static int check_geom(const lq_geom* geom, int min_extent) {
  if (!geom) return fail(LQ_EINVAL, "geometry is NULL");
  for (int k = 0; k < 4; ++k) {
    if (geom->L[k] <= 0 || (geom->L[k] & 1)) return fail(LQ_EINVAL, "lattice extents must be positive and even");
    if (geom->L[k] < min_extent) return fail(LQ_EINVAL, "HISQ needs every extent >= 4 (three-hop Naik term)");
  }
  const int64_t V = (int64_t)geom->L[0] * geom->L[1] * geom->L[2] * geom->L[3];
  if (V / 2 > (int64_t)INT32_MAX / 64) return fail(LQ_EINVAL, "lattice too large");
  return 0;
}

static Geom to_geom(const lq_geom* geom) {
  Geom g{};
  for (int k = 0; k < 4; ++k) g.L[k] = geom->L[k];
  g.Lxh = geom->L[0] / 2;
  g.Vh = (int)((int64_t)geom->L[0] * geom->L[1] * geom->L[2] * geom->L[3] / 2);
  g.ap = geom->t_antiperiodic ? 1 : 0;
  return g;
}

static int check_action(const lq_action* a, const lq_field* f) {
  if (!a) return fail(LQ_EINVAL, "action is NULL");
  if (!f) return fail(LQ_EINVAL, "field is NULL");
  if (a->kind < LQ_WILSON || a->kind > LQ_OVERLAP) return fail(LQ_EINVAL, "unknown action kind");
  if ((a->kind == LQ_HISQ) != (f->type == 1)) return fail(LQ_EINVAL, "field type does not match the action");
  if (a->kind == LQ_OVERLAP) {
    if (!(a->rho > 0)) return fail(LQ_EINVAL, "overlap: rho must be positive");
    if (a->cheb_N < 1 || a->cheb_N > 100000) return fail(LQ_EINVAL, "overlap: cheb_N out of range");
    if ((a->cheb_a != 0 || a->cheb_b != 0) && !(a->cheb_a > 0 && a->cheb_b > a->cheb_a))
      return fail(LQ_EINVAL, "overlap: need 0 < cheb_a < cheb_b");
    if (a->n_lowmodes < 0 || a->n_lowmodes > 1000) return fail(LQ_EINVAL, "overlap: n_lowmodes out of range");
  }
  if (!std::isfinite(a->m) || !std::isfinite(a->mu) || !std::isfinite(a->c_sw))
    return fail(LQ_EINVAL, "non-finite action parameter");
  return 0;
}

// Device scratch of lq_apply_noalloc (its packed input and output vectors).
// Each device holds one copy for the life of the process; host code uses the
// address hipGetSymbolAddress returns on that device, never the symbol.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mtx;
static void* g_scratch_ptr[kMaxDevices] = {};

// address of `scratch` on `device` (the current device), looked up once per device
static int scratch_setup(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(LQ_EINVAL, "device ordinal out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mtx);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(LQ_EDEVICE, "hipGetSymbolAddress of the allocation-free scratch failed");
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return 0;
}

static int64_t field_doubles(const lq_field* f, int kind, int n_rhs) {
  const int nc = kind == LQ_HISQ ? 3 : 12;
  return (int64_t)n_rhs * 2 * f->g.Vh * nc * 2;
}

}  // namespace lq

using namespace lq;

extern "C" {

const char* lq_last_error(void) { return g_err.c_str(); }
const char* lq_version(void) { return "liblq 0.1 (gfx950)"; }

lq_status lq_init(int device, lq_ctx** ctx) {
  if (!ctx) return (lq_status)fail(LQ_EINVAL, "ctx is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return (lq_status)fail(LQ_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return (lq_status)fail(LQ_EINVAL, "device ordinal out of range");
  if (hipSetDevice(device) != hipSuccess) return (lq_status)fail(LQ_EDEVICE, "hipSetDevice failed");
  // the allocation-free entry point's scratch; a failure here only disables that entry point
  void* scr = nullptr;
  if (scratch_setup(device, &scr)) scr = nullptr;
  auto* c = new lq_ctx();
  c->device = device;
  c->scratch = scr;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return (lq_status)fail(LQ_EDEVICE, "stream creation failed");
  }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
  *ctx = c;
  return LQ_OK;
}

lq_status lq_finalize(lq_ctx* c) {
  if (!c) return (lq_status)fail(LQ_EINVAL, "ctx is NULL");
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  prof_flush(c);
  eig_release(c);
  for (auto e : c->event_pool) hipEventDestroy(e);
  if (c->partial) hipFree(c->partial);
  hipStreamDestroy(c->stream);
  delete c;
  return LQ_OK;
}

static lq_status load_common(lq_ctx* c, const lq_geom* geom, const double* a, const double* b, bool dev,
                             void* stream, int type, lq_field** g) {
  if (!c || !g || !a || (type == 1 && !b)) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  int e = check_geom(geom, type == 1 ? 4 : 2);
  if (e) return (lq_status)e;
  hipSetDevice(c->device);
  auto* f = new lq_field();
  f->ctx = c;
  f->type = type;
  f->g = to_geom(geom);
  const size_t bytes = (size_t)2 * f->g.Vh * 4 * 18 * sizeof(double);
  hipStream_t s = dev ? (hipStream_t)stream : c->stream;
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (hipMalloc(&f->aos, bytes) != hipSuccess || (type == 1 && hipMalloc(&f->aos2, bytes) != hipSuccess)) {
    (void)hipGetLastError();
    if (f->aos) hipFree(f->aos);
    delete f;
    return (lq_status)fail(LQ_ENOMEM, "gauge field allocation");
  }
  if (hipMemcpyAsync(f->aos, a, bytes, kind, s) != hipSuccess ||
      (type == 1 && hipMemcpyAsync(f->aos2, b, bytes, kind, s) != hipSuccess) || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    hipFree(f->aos);
    if (f->aos2) hipFree(f->aos2);
    delete f;
    return (lq_status)fail(LQ_EDEVICE, "gauge field upload");
  }
  *g = f;
  return LQ_OK;
}

lq_status lq_gauge_load(lq_ctx* c, const lq_geom* geom, const double* U, lq_field** g) {
  return load_common(c, geom, U, nullptr, false, nullptr, 0, g);
}
lq_status lq_gauge_load_dev(lq_ctx* c, const lq_geom* geom, const double* U, void* stream, lq_field** g) {
  return load_common(c, geom, U, nullptr, true, stream, 0, g);
}
lq_status lq_hisq_load(lq_ctx* c, const lq_geom* geom, const double* fat, const double* lng, lq_field** g) {
  return load_common(c, geom, fat, lng, false, nullptr, 1, g);
}
lq_status lq_hisq_load_dev(lq_ctx* c, const lq_geom* geom, const double* fat, const double* lng, void* stream,
                           lq_field** g) {
  return load_common(c, geom, fat, lng, true, stream, 1, g);
}

lq_status lq_field_free(lq_field* f) {
  if (!f) return (lq_status)fail(LQ_EINVAL, "field is NULL");
  hipSetDevice(f->ctx->device);
  hipDeviceSynchronize();
  auto fr = [](void* p) {
    if (p) hipFree(p);
  };
  fr(f->aos);
  fr(f->aos2);
  for (auto& a : f->links)
    for (auto p : a) fr(p);
  for (auto p : f->fat) fr(p);
  for (auto p : f->lng) fr(p);
  for (auto& kv : f->clover) {
    for (auto p : kv.second.H) fr(p);
    for (auto p : kv.second.Ainv) fr(p);
  }
  for (auto& kv : f->eig) fr(kv.second.vecs);
  mg_release(f->mg);
  delete f;
  return LQ_OK;
}

static int check_apply(lq_ctx* c, const lq_action* act, const lq_field* g, int prec, int n_rhs, const void* in,
                       const void* out) {
  if (!c) return fail(LQ_EINVAL, "ctx is NULL");
  int e = check_action(act, g);
  if (e) return e;
  if ((prec & ~LQ_PREC_RECON12) != 64 && (prec & ~LQ_PREC_RECON12) != 32 && (prec & ~LQ_PREC_RECON12) != 16)
    return fail(LQ_EINVAL, "prec_bits must be 64, 32 or 16 (optionally | LQ_PREC_RECON12)");
  if (n_rhs < 0) return fail(LQ_EINVAL, "n_rhs must be >= 0");
  if (n_rhs > LQ_MAX_COLUMNS) return fail(LQ_EINVAL, "n_rhs above LQ_MAX_COLUMNS");
  if (n_rhs > 0 && (!in || !out)) return fail(LQ_EINVAL, "NULL field pointer");
  return 0;
}

lq_status lq_apply_dev(lq_ctx* c, const lq_action* act, const lq_field* g, int op, int prec, int n_rhs,
                       const double* in, double* out, void* stream) {
  int e = check_apply(c, act, g, prec, n_rhs, in, out);
  if (e) return (lq_status)e;
  if (n_rhs == 0) return LQ_OK;
  hipSetDevice(c->device);
  return (lq_status)apply_op(c, act, const_cast<lq_field*>(g), op, prec, n_rhs, in, out, (hipStream_t)stream);
}

lq_status lq_apply_noalloc(lq_ctx* c, const lq_action* act, const lq_field* g, int op, int prec, int n_rhs,
                           const double* in, double* out, void* stream) {
  int e = check_apply(c, act, g, prec, n_rhs, in, out);
  if (e) return (lq_status)e;
  if (n_rhs == 0) return LQ_OK;
  hipSetDevice(c->device);
  return (lq_status)apply_op_noalloc(c, act, const_cast<lq_field*>(g), op, prec, n_rhs, in, out, (hipStream_t)stream,
                                     c->scratch, kNoallocScratchBytes);
}

lq_status lq_apply(lq_ctx* c, const lq_action* act, const lq_field* g, int op, int prec, int n_rhs, const double* in,
                   double* out) {
  int e = check_apply(c, act, g, prec, n_rhs, in, out);
  if (e) return (lq_status)e;
  if (n_rhs == 0) return LQ_OK;
  hipSetDevice(c->device);
  const size_t bytes = sizeof(double) * field_doubles(g, act->kind, n_rhs);
  DBuf din(bytes, c->stream), dout(bytes, c->stream);
  if (!din.p || !dout.p) return (lq_status)fail(LQ_ENOMEM, "staging buffers");
  if (hipMemcpyAsync(din.p, in, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return (lq_status)fail(LQ_EDEVICE, "upload");
  e = apply_op(c, act, const_cast<lq_field*>(g), op, prec, n_rhs, din.as<double>(), dout.as<double>(), c->stream);
  if (e) return (lq_status)e;
  if (hipMemcpyAsync(out, dout.p, bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return (lq_status)fail(LQ_EDEVICE, "download");
  return LQ_OK;
}

static int check_solve(lq_ctx* c, const lq_action* act, const lq_field* g, const lq_params* prm, int n_rhs,
                       const void* b, const void* x) {
  if (!c || !prm) return fail(LQ_EINVAL, "NULL argument");
  int e = check_action(act, g);
  if (e) return e;
  if (n_rhs < 0) return fail(LQ_EINVAL, "n_rhs must be >= 0");
  if (n_rhs > 0 && (!b || !x)) return fail(LQ_EINVAL, "NULL field pointer");
  if (prm->sloppy_bits != 0 && prm->sloppy_bits != 16 && prm->sloppy_bits != 32 && prm->sloppy_bits != 64)
    return fail(LQ_EINVAL, "sloppy_bits must be 64, 32 or 16");
  if (!(prm->tol >= 0) || prm->tol >= 1.0) return fail(LQ_EINVAL, "tol must be in [0, 1)");
  if (prm->n_shift < 0 || prm->n_shift > 64) return fail(LQ_EINVAL, "n_shift out of range");
  {
    // columns the solver carries: the masses, and the overlap solve's two chiral sectors
    const int64_t cols = (int64_t)n_rhs * (prm->n_shift > 1 ? prm->n_shift : 1) *
                         (act->kind == LQ_OVERLAP && prm->solver == 0 ? 2 : 1);
    if (cols > LQ_MAX_COLUMNS)
      return fail(LQ_EINVAL, "n_rhs (x n_shift, x 2 for the overlap sectors) above LQ_MAX_COLUMNS");
  }
  if (prm->n_shift > 1 && act->kind != LQ_HISQ && act->kind != LQ_OVERLAP)
    return fail(LQ_EINVAL, "several masses are implemented for HISQ and overlap");
  if (prm->solver < 0 || prm->solver > 3) return fail(LQ_EINVAL, "solver must be 0, 1, 2 or 3");
  if ((prm->solver == 2 || prm->solver == 3) && act->kind != LQ_TM_CLOVER)
    return fail(LQ_EINVAL, "solvers 2 (GCR) and 3 (multigrid) are implemented for the twisted-clover action");
  if (prm->n_shift > 1 && act->kind == LQ_OVERLAP && prm->solver == 1)
    return fail(LQ_EINVAL, "overlap: several masses need the chirally projected solver (solver = 0)");
  return 0;
}

static size_t solution_doubles(const lq_field* g, const lq_action* act, const lq_params* prm, int n_rhs) {
  const int nsh = ((act->kind == LQ_HISQ || act->kind == LQ_OVERLAP) && prm->n_shift > 1) ? prm->n_shift : 1;
  return (size_t)nsh * field_doubles(g, act->kind, n_rhs);
}

lq_status lq_solve_dev(lq_ctx* c, const lq_action* act, const lq_field* g, const lq_params* prm, int n_rhs,
                       const double* b, double* x, lq_stats* st, void* stream) {
  int e = check_solve(c, act, g, prm, n_rhs, b, x);
  if (e) return (lq_status)e;
  if (st) std::memset(st, 0, sizeof(*st));
  if (n_rhs == 0) return LQ_OK;
  hipSetDevice(c->device);
  e = solve(c, act, const_cast<lq_field*>(g), prm, n_rhs, b, x, st, (hipStream_t)stream);
  if (st) st->status = e;
  return (lq_status)e;
}

lq_status lq_solve(lq_ctx* c, const lq_action* act, const lq_field* g, const lq_params* prm, int n_rhs,
                   const double* b, double* x, lq_stats* st) {
  int e = check_solve(c, act, g, prm, n_rhs, b, x);
  if (e) return (lq_status)e;
  if (st) std::memset(st, 0, sizeof(*st));
  if (n_rhs == 0) return LQ_OK;
  hipSetDevice(c->device);
  const size_t nb = sizeof(double) * field_doubles(g, act->kind, n_rhs);
  const size_t nx = sizeof(double) * solution_doubles(g, act, prm, n_rhs);
  DBuf db(nb, c->stream), dx(nx, c->stream);
  if (!db.p || !dx.p) return (lq_status)fail(LQ_ENOMEM, "staging buffers");
  if (hipMemcpyAsync(db.p, b, nb, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      (prm->use_initial_guess && hipMemcpyAsync(dx.p, x, nx, hipMemcpyHostToDevice, c->stream) != hipSuccess))
    return (lq_status)fail(LQ_EDEVICE, "upload");
  e = solve(c, act, const_cast<lq_field*>(g), prm, n_rhs, db.as<double>(), dx.as<double>(), st, c->stream);
  if (st) st->status = e;
  if (e != LQ_OK && e != LQ_ENOCONV && e != LQ_EBREAKDOWN) return (lq_status)e;
  const std::string msg = g_err;
  if (hipMemcpyAsync(x, dx.p, nx, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return (lq_status)fail(LQ_EDEVICE, "download");
  g_err = msg;
  return (lq_status)e;
}

lq_status lq_eigs(lq_ctx* c, const lq_action* act, const lq_field* g, int which, int nev, double tol,
                  int max_restarts, int filter_degree, double filter_cut, double* evals, lq_stats* stats) {
  if (!c) return (lq_status)fail(LQ_EINVAL, "ctx is NULL");
  int e = check_action(act, g);
  if (e) return (lq_status)e;
  if (act->kind != LQ_OVERLAP) return (lq_status)fail(LQ_EINVAL, "lq_eigs needs the overlap action");
  if (!(act->rho > 0)) return (lq_status)fail(LQ_EINVAL, "lq_eigs: rho must be positive");
  hipSetDevice(c->device);
  return (lq_status)eigs(c, act, const_cast<lq_field*>(g), which, nev, tol, max_restarts, filter_degree, filter_cut,
                         evals, stats, c->stream);
}

lq_status lq_hw_bounds(lq_ctx* c, const lq_action* act, const lq_field* g, int iters, double* lmin, double* lmax) {
  if (!c || !act || !g || !lmin || !lmax) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  if (g->type != 0) return (lq_status)fail(LQ_EINVAL, "H_W bounds need a Wilson gauge field");
  if (iters < 2) iters = 200;
  hipSetDevice(c->device);
  int e = hw_bounds(c, act, const_cast<lq_field*>(g), iters, lmin, lmax, c->stream);
  if (!e && hipStreamSynchronize(c->stream) != hipSuccess) e = fail(LQ_EDEVICE, "sync");
  return (lq_status)e;
}

lq_status lq_mg_setup(lq_ctx* c, const lq_action* act, const lq_field* g, const lq_mg_params* mp, lq_stats* stats) {
  if (!c) return (lq_status)fail(LQ_EINVAL, "ctx is NULL");
  int e = check_action(act, g);
  if (e) return (lq_status)e;
  hipSetDevice(c->device);
  return (lq_status)mg_setup(c, act, const_cast<lq_field*>(g), mp, stats, c->stream);
}

lq_status lq_mg_apply(lq_ctx* c, const lq_action* act, const lq_field* g, int op, int prec, int n_rhs, const double* in,
                      double* out) {
  if (!c) return (lq_status)fail(LQ_EINVAL, "ctx is NULL");
  int e = check_action(act, g);
  if (e) return (lq_status)e;
  if (n_rhs < 0) return (lq_status)fail(LQ_EINVAL, "n_rhs must be >= 0");
  if (n_rhs > LQ_MAX_COLUMNS) return (lq_status)fail(LQ_EINVAL, "n_rhs above LQ_MAX_COLUMNS");
  if (n_rhs > 0 && (!in || !out)) return (lq_status)fail(LQ_EINVAL, "NULL array");
  hipSetDevice(c->device);
  return (lq_status)mg_apply_host(c, act, const_cast<lq_field*>(g), op, prec, n_rhs, in, out, c->stream);
}

lq_status lq_cheb_coeffs(double a, double b, int N, double* c) {
  if (!c || N < 0 || !(a > 0) || !(b > a)) return (lq_status)fail(LQ_EINVAL, "need 0 < a < b, N >= 0, c != NULL");
  cheb_coeffs(a, b, N, c);
  return LQ_OK;
}

lq_status lq_copy_bandwidth(lq_ctx* c, size_t bytes, int reps, double* gbs) {
  if (!c || !gbs || bytes < 16 || reps < 1) return (lq_status)fail(LQ_EINVAL, "need ctx, gbs, bytes >= 16, reps >= 1");
  hipSetDevice(c->device);
  bytes = bytes / 16 * 16;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (a) hipFree(a);
    return (lq_status)fail(LQ_ENOMEM, "copy buffers");
  }
  hipStream_t s = c->stream;
  int e = launch_fill_zero(a, bytes, s) || launch_stream_copy(a, b, bytes, s);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipEventRecord(e0, s);
  for (int k = 0; k < reps && !e; ++k) {
    Prof p(c, "stream_copy", s);
    e = launch_stream_copy(a, b, bytes, s);
  }
  hipEventRecord(e1, s);
  hipEventSynchronize(e1);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(a);
  hipFree(b);
  if (e) return (lq_status)fail(LQ_EDEVICE, "copy kernel");
  *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
  return LQ_OK;
}

lq_status lq_profile(lq_ctx* c, int enable) {
  if (!c) return (lq_status)fail(LQ_EINVAL, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> lk(c->prof_mtx);
  prof_flush(c);
  if (enable) {
    c->totals.clear();
    c->byte_totals.clear();
  }
  c->prof = enable != 0;
  return LQ_OK;
}

lq_status lq_profile_bytes(lq_ctx* c, const char* name, double* bytes) {
  if (!c || !name || !bytes) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> lk(c->prof_mtx);
  prof_flush(c);
  auto it = c->byte_totals.find(name);
  *bytes = it == c->byte_totals.end() ? 0.0 : it->second;
  return LQ_OK;
}

lq_status lq_profile_get(lq_ctx* c, const char* name, int64_t* count, double* avg_ms) {
  if (!c || !name || !count || !avg_ms) return (lq_status)fail(LQ_EINVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> lk(c->prof_mtx);
  prof_flush(c);
  auto it = c->totals.find(name);
  if (it == c->totals.end()) {
    *count = 0;
    *avg_ms = 0;
    return LQ_OK;
  }
  *count = it->second.first;
  *avg_ms = it->second.first ? it->second.second / it->second.first : 0.0;
  return LQ_OK;
}

}  // extern "C"
