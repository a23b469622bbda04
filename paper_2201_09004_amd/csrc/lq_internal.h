// Host-side objects of liblq: context, fields, device vectors, kernel timing,
// and the operator / solver entry points used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lq.h"
#include "lq_kernels.h"

namespace lq {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

inline int pidx(int prec) { return prec == 64 ? 0 : prec == 32 ? 1 : 2; }

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
  double bytes;  // algorithmic bytes of the work timed
};

// tuned launch shape of a stencil kernel
struct Shape {
  int nr;    // columns per thread
  int slab;  // traversal slab depth (0: lexicographic)
  int tpb;   // site tiles per workgroup (0: automatic)
  int xcd;   // XCD-aware block order
};

}  // namespace lq

struct lq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // stream of the host-pointer API
  std::atomic<bool> prof{false};
  std::vector<lq::ProfRec> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, std::pair<int64_t, double>> totals;
  std::map<std::string, double> byte_totals;  // algorithmic bytes per timed name
  void* scratch = nullptr;    // this device's address of the allocation-free entry point's scratch
  void* rocblas = nullptr;    // rocBLAS handle of the eigensolver (created on first use)
  double* partial = nullptr;  // reduction partials
  size_t partial_bytes = 0;
  std::mutex mtx;
  std::recursive_mutex prof_mtx;  // kernel timing records (shared by API threads and the server worker)
  // autotuned launch shapes per kernel key
  std::map<std::string, lq::Shape> tune;
  bool tune_loaded = false;
};

namespace lq {

struct Clover {
  void* H[2] = {nullptr, nullptr};     // [FP64, FP32] packed Hermitian (4+m)+C
  void* Ainv[2] = {nullptr, nullptr};  // [FP64, FP32] full complex (H +- i mu)^{-1}
};

// Lanczos estimate of the spectrum of H_W^2: extreme Ritz values and the FP64
// residual norms of their Ritz vectors
struct HwSpectrum {
  double theta_min, theta_max, r_min, r_max;
  int steps;
};

// Resident low modes of a field: eigenvectors (FP64 Wilson-type columns, both
// parities, make_vec layout) of H_W (which = LQ_EIG_HW, chir = 0) or of the
// chiral-sector overlap operator (LQ_EIG_OVERLAP, chir = +-1) for one rho
struct EigSet {
  int which = 0, chir = 0, n = 0;
  double rho = 0;
  void* vecs = nullptr;
  std::vector<double> vals, res;  // eigenvalues (H_W: ascending |lambda|; sector: ascending) and residuals
};

// Two-level aggregation multigrid hierarchy of a field for one Wilson-type
// action: aggregate maps, the chirality-split orthonormal basis Q and the
// Galerkin coarse operator Dc (FP64 and FP32 copies), and the V-cycle settings
struct MgHier {
  int kind = 0;
  double m = 0, mu = 0, csw = 0;  // action the hierarchy was built for
  int block[4] = {0, 0, 0, 0}, Lc[4] = {0, 0, 0, 0};
  int Vc = 0, B = 0, nv = 0, K = 0;
  int *fine = nullptr, *nbr = nullptr, *face = nullptr, *cpar = nullptr, *cmap = nullptr, *csite = nullptr;
  std::vector<int> cmap_h;  // host copy of cmap
  void *Q64 = nullptr, *Q32 = nullptr, *Dc64 = nullptr, *Dc32 = nullptr;
  // A^{-1} (direction 0) and A^{-1} Dc[d] (d = 1..8) of every aggregate: the
  // even-odd preconditioned coarse operator
  void *Ahat64 = nullptr, *Ahat32 = nullptr;
  Geom gc{};  // shape of coarse vectors: Vh = K * Vc / 2 pseudo-sites per coarse parity
  double coarse_tol = 0.1;
  int coarse_maxiter = 100, nu_post = 4, gcr_kmax = 8, nu_pre = 0;
  double setup_seconds = 0;
  int setup_iters = 0;
  MgGeom geom() const { return MgGeom{Vc, B, nv, K, fine, nbr, face, cpar, cmap, csite}; }
};

}  // namespace lq

struct lq_field {
  lq_ctx* ctx = nullptr;
  int type = 0;  // 0 Wilson gauge, 1 HISQ
  lq::Geom g{};
  double* aos = nullptr;   // canonical FP64 copy (gauge / fat)
  double* aos2 = nullptr;  // long links
  void* links[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  void* fat[3] = {nullptr, nullptr, nullptr};
  void* lng[3] = {nullptr, nullptr, nullptr};
  float sfat[3] = {1, 1, 1}, slng[3] = {1, 1, 1};
  std::map<std::tuple<double, double, double>, lq::Clover> clover;
  std::map<double, lq::HwSpectrum> hw_spec;  // per rho: Lanczos spectrum of H_W^2
  std::map<std::tuple<int, double, int>, lq::EigSet> eig;  // (which, rho, chirality): low modes
  lq::MgHier* mg = nullptr;  // multigrid hierarchy (lq_mg_setup), one per field
  std::mutex mtx;
};

namespace lq {

// ------------------------------------------------------------------ timing
// Times the work enqueued on stream st during its lifetime (when profiling is
// on).  The record joins the context's pending list only once its end event
// is recorded, so flushing the list never touches a record still in use.
struct Prof {
  lq_ctx* c;
  hipStream_t s;
  bool on = false;
  ProfRec rec;
  Prof(lq_ctx* ctx, const char* name, hipStream_t st, double bytes = 0.0);
  ~Prof();
  Prof(const Prof&) = delete;
  Prof& operator=(const Prof&) = delete;
};
void prof_flush(lq_ctx* c);

// ------------------------------------------------------------------ vectors
// A set of ncol columns of one field type (nc = 12 Wilson, 3 staggered) and
// precision, storing npar parities per column (npar = 1: parity `par0` only).
struct Vec {
  FieldRef f{};
  int prec = 64, nc = 12, ncol = 0, npar = 2, par0 = 0;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  bool owner = true;
  Vec() = default;
  Vec(const Vec&) = delete;
  Vec& operator=(const Vec&) = delete;
  Vec(Vec&& o) noexcept { *this = std::move(o); }
  Vec& operator=(Vec&& o) noexcept;
  ~Vec();
  bool ok() const { return f.data != nullptr || ncol == 0; }
  // view of columns [c0, c0+n)
  FieldRef cols(int c0) const;
};
Vec make_vec(const Geom& g, int prec, int nc, int ncol, int npar, int par0, hipStream_t s);
Vec view(const Vec& v, int c0, int n);  // non-owning view of columns [c0, c0+n)
int vec_zero(Vec& v);
int vec_copy(Vec& dst, const Vec& src);  // with precision conversion, same shape
int vec_swap_cols(Vec& v, int a, int b);  // exchange columns a and b in place
// bytes make_vec allocates for this shape, and a non-owning Vec over `base`
size_t vec_bytes(const Geom& g, int prec, int nc, int ncol, int npar);
Vec vec_at(const Geom& g, int prec, int nc, int ncol, int npar, int par0, void* base, hipStream_t s);

// scoped device buffer
struct DBuf {
  void* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  DBuf() = default;
  DBuf(size_t bytes, hipStream_t st);
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      if (p) hipFreeAsync(p, s);
      p = o.p;
      n = o.n;
      s = o.s;
      o.p = nullptr;
    }
    return *this;
  }
  ~DBuf();
  template <typename T> T* as() const { return (T*)p; }
};

// ------------------------------------------------------------------ operators
struct OpEnv {
  lq_ctx* ctx;
  lq_field* f;
  lq_action act;
  hipStream_t s;
  int recon = 0;
  std::vector<double> cheb;  // Chebyshev coefficients (overlap)
  double a = 0, b = 0;
  int64_t n_apply = 0;       // stencil half-applications (counted per parity)
  double flops = 0, bytes = 0;
  bool noalloc = false;      // no device allocation: fields must be resident, shapes are not tuned
};

int ensure_links(OpEnv& e, int prec);
int ensure_clover(OpEnv& e, int prec);
const Clover* get_clover(OpEnv& e);

// Wilson-type: full-lattice D, D^dag, hop; site terms; Schur operator and helpers
int wilson_D(OpEnv& e, int prec, Vec& out, const Vec& in, bool dag);
int wilson_hop(OpEnv& e, int prec, Vec& out, const Vec& in);
int tm_site(OpEnv& e, int prec, Vec& out, const Vec& in, bool inverse);
// red_mode 2: the partials of <out, in> and |out|^2 are written to red as
// [col][64-site tiles of Vh][4] by the second stencil (EPI_XMY_RTS)
int tm_schur(OpEnv& e, int prec, Vec& out_e, const Vec& in_e, Vec& tmp_o, int red_mode = 0, double* red = nullptr);
int tm_schur_source(OpEnv& e, Vec& bhat_e, const Vec& b);                 // in b's precision
int tm_schur_reconstruct(OpEnv& e, Vec& x, const Vec& x_e, const Vec& b); // x full; all in x's precision
// overlap
int hw_apply(OpEnv& e, int prec, Vec& out, const Vec& in);
int sign_apply(OpEnv& e, int prec, Vec& out, const Vec& in);
// Chebyshev filter T_d(Z(H_W^2)) v, Z = (2 H_W^2 - (lo + hi)) / (hi - lo), FP64
int cheb_filter(OpEnv& e, Vec& out, const Vec& in, double lo, double hi, int d);
int overlap_D(OpEnv& e, int prec, Vec& out, const Vec& in, bool dag);
int overlap_prepare(OpEnv& e);
// staggered
int stag_D(OpEnv& e, int prec, Vec& out, const Vec& in, bool dag, const double* acol_dev = nullptr);
int stag_hop(OpEnv& e, int prec, Vec& out, const Vec& in);
// red: if not null, <in_e, out_e> per column as partials over 64-site tiles
// ([col][tile][4], re and im in the first two) from the second stencil's epilogue
int stag_normal_even(OpEnv& e, int prec, Vec& out_e, const Vec& in_e, Vec& tmp_o, const double* acol_dev, double a,
                     double* red = nullptr);

// ------------------------------------------------------------------ BLAS helpers
struct Blas {
  lq_ctx* ctx = nullptr;
  hipStream_t s = nullptr;
  int gridx = 1;
  double* partial = nullptr;  // owned by `part`, sized for the columns given to blas_prepare
  DBuf part;
  int op(int opc, Vec* f0, Vec* f1 = nullptr, Vec* f2 = nullptr, Vec* f3 = nullptr, Vec* f4 = nullptr,
         const double* st = nullptr, int c0 = 0, int c1 = 0);
  int opi(int opc, Vec* f0, Vec* f1, Vec* f2, double c0re, double c0im = 0, double c1re = 0, double c1im = 0);
  // OP_PLC: f2 = p0 f0 + p1 (p2 f1 + p3 g5 f1) with [ncol][4] coefficients pcol (device)
  int plc(Vec* f0, Vec* f1, Vec* f2, const double* pcol);
};
int blas_prepare(lq_ctx* c, Blas& b, const Geom& g, int npar, int ncol, hipStream_t s);

int solve(lq_ctx* c, const lq_action* act, lq_field* f, const lq_params* prm, int n_rhs, const double* b_dev,
          double* x_dev, lq_stats* st, hipStream_t s);
int apply_op(lq_ctx* c, const lq_action* act, lq_field* f, int op, int prec, int n_rhs, const double* in_dev,
             double* out_dev, hipStream_t s);
// apply_op for D, D^dag, the hopping term and H_W with its packed vectors in
// `scratch` (scratch_bytes long) and no device allocation; enqueue only
int apply_op_noalloc(lq_ctx* c, const lq_action* act, lq_field* f, int op, int prec, int n_rhs,
                     const double* in_dev, double* out_dev, hipStream_t s, void* scratch, size_t scratch_bytes);
int hw_spectrum(lq_ctx* c, const lq_action* act, lq_field* f, int iters, HwSpectrum* out, hipStream_t s);
// certified interval: lmin^2 = theta_min - r_min, lmax^2 = theta_max + r_max
int hw_bounds(lq_ctx* c, const lq_action* act, lq_field* f, int iters, double* lmin, double* lmax, hipStream_t s);
void cheb_coeffs(double a, double b, int N, double* c);

// low modes (eig.cpp)
int eigs(lq_ctx* c, const lq_action* act, lq_field* f, int which, int nev, double tol, int max_restarts, int degree,
         double cut, double* evals, lq_stats* st, hipStream_t s);
const EigSet* find_eigs(lq_field* f, int which, double rho, int chir);
// v <- (1 - U U^H) v over the first n modes; coef (device, n x v.ncol complex) <- U^H v
int project_out(lq_ctx* c, const Geom& g, hipStream_t s, const EigSet& es, int n, Vec& v, void* coef);
// v += U diag(w) coef, w[col * n + i] (host)
int add_modes(lq_ctx* c, const Geom& g, hipStream_t s, const EigSet& es, int n, const std::vector<double>& w,
              Vec& v, void* coef);
void eig_release(lq_ctx* c);

// multigrid (mg.cpp; setup and solve in solvers.cpp)
int mg_init_maps(MgHier& h, const Geom& g, const int block[4], int nv);
int mg_build(OpEnv& e, MgHier& h, Vec& vecs);  // basis from vecs (FP64, nv columns), then Dc
void mg_release(MgHier* h);
int mg_restrict(OpEnv& e, const MgHier& h, const Vec& fine, Vec& coarse);
int mg_prolong(OpEnv& e, const MgHier& h, const Vec& coarse, Vec& fine);
int mg_coarse_op(OpEnv& e, const MgHier& h, Vec& out, const Vec& in);
// even-odd coarse system: bhat_e = A_ee^-1 (b_e - D_eo A_oo^-1 b_o) with t_o = A_oo^-1 b_o kept,
// out_e = (1 - A_ee^-1 D_eo A_oo^-1 D_oe) in_e, x_o = t_o - A_oo^-1 D_oe x_e (x full, x_e copied in)
int mg_schur_source(OpEnv& e, const MgHier& h, Vec& bhat_e, Vec& t_o, Vec& u_e, const Vec& b);
int mg_schur_op(OpEnv& e, const MgHier& h, Vec& out_e, const Vec& in_e, Vec& tmp_o);
int mg_schur_reconstruct(OpEnv& e, const MgHier& h, Vec& x, const Vec& x_e, const Vec& t_o);
int mg_apply_host(lq_ctx* c, const lq_action* act, lq_field* f, int op, int prec, int n_rhs, const double* in,
                  double* out, hipStream_t s);
int mg_setup(lq_ctx* c, const lq_action* act, lq_field* f, const lq_mg_params* mp, lq_stats* st, hipStream_t s);
bool mg_matches(const MgHier* h, const lq_action* act);
// the setup's probe vectors on the fine lattice (FP64, ncol <= 12 columns): basis vector
// (k0 + kk) of the aggregates of coarse parity class cls in column kk, zero elsewhere (mg.hip)
int launch_mg_probe_fine(const MgGeom& m, const void* Q64, FieldRef fine, int ncol, int k0, int cls, hipStream_t s);
// one classical Gram-Schmidt step over k <= 8 directions (mg.hip): coef[j][col] = <W_j, w>,
// then w -= sum_j coef_j W_j and z -= sum_j coef_j Z_j; partial holds k * ncol * gridx * 2 doubles
int launch_mg_cgs(int prec, const FieldRef* W, const FieldRef* Z, int k, FieldRef w, FieldRef z, int ncol, int npar,
                  int gridx, double* partial, double* coef, hipStream_t s);

}  // namespace lq
