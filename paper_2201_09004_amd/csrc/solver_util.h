// Host helpers shared by the Krylov drivers and the serving engines:
// pinned host buffers, device-resident per-column solver state with its host
// mirror, per-column norms and FP64 true residuals.
#pragma once

#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "lq_internal.h"

namespace lq {

struct HostPinned {
  double* p = nullptr;
  explicit HostPinned(size_t n) {
    if (hipHostMalloc((void**)&p, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
  ~HostPinned() {
    if (p) hipHostFree(p);
  }
};

// per-column solver state [ncol][ST_STRIDE] on the device and in pinned host memory
struct State {
  DBuf dev;
  HostPinned host;
  int ncol;
  hipStream_t s;
  State(int n, hipStream_t st)
      : dev((size_t)std::max(n, 1) * ST_STRIDE * 8, st), host((size_t)std::max(n, 1) * ST_STRIDE), ncol(n), s(st) {}
  bool ok() const { return dev.p && host.p; }
  double* d() { return dev.as<double>(); }
  double& h(int col, int k) { return host.p[col * ST_STRIDE + k]; }
  int pull(int n = -1) {
    const size_t cnt = (size_t)(n < 0 ? ncol : n) * ST_STRIDE * 8;
    if (hipMemcpyAsync(host.p, dev.p, cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LQ_EDEVICE, "state readback");
    return 0;
  }
  int push(int n = -1) {
    const size_t cnt = (size_t)(n < 0 ? ncol : n) * ST_STRIDE * 8;
    if (hipMemcpyAsync(dev.p, host.p, cnt, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(LQ_EDEVICE, "state upload");
    return 0;
  }
};

using OpFn = std::function<int(Vec& out, const Vec& in)>;

// Reliable-update trigger for a batch of columns.  A column is due once its
// iterated residual has dropped by delta since the last update; the batch
// recomputes its FP64 residuals when a column may have converged, when one
// column has dropped by delta^2 (its recursion error is then about the
// sloppy precision times 1/delta^2 of its residual), or when half of the
// active columns are due.  One update then serves every column.
struct UpdateRule {
  int due = 0, active = 0;
  int conv = 0;        // columns whose iterated residual is below their target
  bool drop = false;   // a column dropped by delta^2 since its last update
  bool now = false;
  void column(double rr, double maxrr, double tol2bb, double delta) {
    ++active;
    const double d2 = delta * delta;
    if (rr < tol2bb) ++conv;
    if (rr < d2 * d2 * maxrr) drop = true;
    if (rr < tol2bb || rr < d2 * d2 * maxrr) now = true;
    else if (rr < d2 * maxrr) ++due;
  }
  bool fire() const { return now || (active > 0 && 2 * due >= active); }
  // the update is due only because a few columns may have converged: checking
  // those columns alone is enough
  bool converged_few() const { return conv > 0 && !drop && 2 * due < active && 4 * conv <= active; }
};

// Iterations until a column's squared residual rr reaches the next threshold
// of UpdateRule (due at delta^2 maxrr, then convergence or delta^4 maxrr),
// predicted from its mean reduction per iteration since the previous host
// check (rr_prev, steps iterations ago); 0 when it is not decreasing.  A
// solver that reads its state every iteration only to evaluate the rule can
// skip the reads for about half the smallest such count.
inline double iters_to_event(double rr, double rr_prev, int steps, double maxrr, double tol2bb, double delta) {
  const double d2 = delta * delta;
  const double t = std::max(tol2bb, rr >= d2 * maxrr ? d2 * maxrr : d2 * d2 * maxrr);
  if (!(rr > t) || !(rr_prev > 0.0) || steps <= 0) return 0.0;
  const double f = std::pow(rr / rr_prev, 1.0 / steps);
  if (!(f < 0.999)) return 0.0;
  return std::log(t / rr) / std::log(f);
}

// per-column |v|^2 (host vector)
int col_norms(Blas& bl, Vec& v, std::vector<double>& out);
// per-column relative residual |b - A x| / |b| in FP64
int rel_residual(Blas& bl, const OpFn& A, Vec& x, Vec& b, std::vector<double>& res, const Geom& g);

}  // namespace lq
