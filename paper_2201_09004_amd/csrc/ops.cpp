// Operators of the four actions composed from the stencil, site and BLAS
// kernels: Wilson and twisted-clover D (sec. 2.1), the even-odd Schur
// complement, H_W and the Chebyshev/Clenshaw sign function with the overlap
// operator (sec. 2.3), and the HISQ staggered operator with its even-site
// normal operator (sec. 2.2).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "lq_internal.h"

namespace lq {

// ------------------------------------------------------------------ timing
Prof::Prof(lq_ctx* ctx, const char* name, hipStream_t st, double bytes) : c(ctx), s(st) {
  if (!c || !c->prof) return;
  std::lock_guard<std::recursive_mutex> lk(c->prof_mtx);
  hipEvent_t ev[2];
  for (int k = 0; k < 2; ++k) {
    if (!c->event_pool.empty()) {
      ev[k] = c->event_pool.back();
      c->event_pool.pop_back();
    } else if (hipEventCreate(&ev[k]) != hipSuccess) {
      (void)hipGetLastError();
      if (k == 1) c->event_pool.push_back(ev[0]);
      return;
    }
  }
  rec = {name, ev[0], ev[1], bytes};
  on = hipEventRecord(ev[0], s) == hipSuccess;
  if (!on) {
    (void)hipGetLastError();
    c->event_pool.push_back(ev[0]);
    c->event_pool.push_back(ev[1]);
  }
}
Prof::~Prof() {
  if (!on) return;
  std::lock_guard<std::recursive_mutex> lk(c->prof_mtx);
  if (hipEventRecord(rec.b, s) != hipSuccess) {
    (void)hipGetLastError();
    c->event_pool.push_back(rec.a);
    c->event_pool.push_back(rec.b);
    return;
  }
  c->pending.push_back(rec);
  if (c->pending.size() > 8192) prof_flush(c);
}
void prof_flush(lq_ctx* c) {
  std::lock_guard<std::recursive_mutex> lk(c->prof_mtx);
  for (auto& r : c->pending) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
    auto& t = c->totals[r.name];
    t.first += 1;
    t.second += ms;
    c->byte_totals[r.name] += r.bytes;
    c->event_pool.push_back(r.a);
    c->event_pool.push_back(r.b);
  }
  c->pending.clear();
}

// field transfers of one BLAS op per site and column (each operand read
// once, each result written once): its algorithmic bytes for the timing records
static int blas_transfers(int op) {
  switch (op) {
    case OP_AXPY: case OP_AXMY: case OP_XPAY: case OP_XMY_NORM: case OP_LC_G5: case OP_PLC: return 3;
    case OP_CG: return 6;
    case OP_BICG_XR: return 7;
    case OP_BICG_P: return 4;
    case OP_DOT: case OP_DOT_NORM: case OP_SCALE: case OP_G5: case OP_COPY: return 2;
    default: return 1;
  }
}
static const char* blas_name(int op) {
  static const char* n[] = {"axpy", "axmy", "xpay", "cg", "bicg_xr", "bicg_p", "dot", "norm2", "dot_norm",
                            "xmy_norm", "zero", "scale", "g5", "lc_g5", "copy", "plc"};
  return op >= 0 && op < OP_NCOUNT ? n[op] : "op";
}
struct BlasProf {
  Prof all, one;
  char name[48];
  static double bytes(const BlasArgs& A) {
    return (double)A.ncol * A.npar * A.Vh * blas_transfers(A.op) * (site_bytes(A.prec, A.nc) + (sep_norm(A.prec, A.nc) ? 4 : 0));
  }
  BlasProf(lq_ctx* c, const BlasArgs& A, hipStream_t s)
      : all(c, "blas", s, bytes(A)), one(c, (snprintf(name, sizeof(name), "blas%d_%s", A.prec, blas_name(A.op)), name),
                                         s, bytes(A)) {}
};

// ------------------------------------------------------------------ vectors
static size_t block_bytes(int prec, int nc, int Vh) { return (size_t)site_bytes(prec, nc) * Vh; }

Vec make_vec(const Geom& g, int prec, int nc, int ncol, int npar, int par0, hipStream_t s) {
  Vec v;
  v.prec = prec;
  v.nc = nc;
  v.ncol = ncol;
  v.npar = npar;
  v.par0 = par0;
  v.s = s;
  const size_t nblk = (size_t)ncol * npar;
  const size_t main = nblk * block_bytes(prec, nc, g.Vh);
  const size_t nb = sep_norm(prec, nc) ? nblk * g.Vh * sizeof(float) : 0;
  const size_t mainr = (main + 255) / 256 * 256;
  v.bytes = mainr + nb;
  v.f.npar = npar;
  v.f.Vh = g.Vh;
  if (ncol == 0) return v;
  void* p = nullptr;
  if (hipMallocAsync(&p, v.bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return v;
  }
  v.f.data = p;
  v.f.norm = sep_norm(prec, nc) ? (float*)((char*)p + mainr) : nullptr;
  return v;
}

size_t vec_bytes(const Geom& g, int prec, int nc, int ncol, int npar) {
  const size_t nblk = (size_t)ncol * npar;
  const size_t main = nblk * block_bytes(prec, nc, g.Vh);
  const size_t nb = sep_norm(prec, nc) ? nblk * g.Vh * sizeof(float) : 0;
  return (main + 255) / 256 * 256 + nb;
}

Vec vec_at(const Geom& g, int prec, int nc, int ncol, int npar, int par0, void* base, hipStream_t s) {
  Vec v;
  v.prec = prec;
  v.nc = nc;
  v.ncol = ncol;
  v.npar = npar;
  v.par0 = par0;
  v.s = s;
  v.owner = false;
  v.bytes = vec_bytes(g, prec, nc, ncol, npar);
  v.f.npar = npar;
  v.f.Vh = g.Vh;
  if (ncol == 0) return v;
  const size_t main = (size_t)ncol * npar * block_bytes(prec, nc, g.Vh);
  v.f.data = base;
  v.f.norm = sep_norm(prec, nc) ? (float*)((char*)base + (main + 255) / 256 * 256) : nullptr;
  return v;
}

Vec& Vec::operator=(Vec&& o) noexcept {
  if (this != &o) {
    if (f.data && owner) hipFreeAsync(f.data, s);
    f = o.f;
    prec = o.prec;
    nc = o.nc;
    ncol = o.ncol;
    npar = o.npar;
    par0 = o.par0;
    bytes = o.bytes;
    s = o.s;
    owner = o.owner;
    o.f.data = nullptr;
    o.f.norm = nullptr;
  }
  return *this;
}
Vec::~Vec() {
  if (f.data && owner) hipFreeAsync(f.data, s);
}
Vec view(const Vec& v, int c0, int n) {
  Vec r;
  r.f = v.cols(c0);
  r.prec = v.prec;
  r.nc = v.nc;
  r.ncol = n;
  r.npar = v.npar;
  r.par0 = v.par0;
  r.s = v.s;
  r.owner = false;
  r.bytes = 0;
  return r;
}
FieldRef Vec::cols(int c0) const {
  FieldRef r = f;
  const size_t nblk = (size_t)c0 * npar;
  r.data = (char*)f.data + nblk * block_bytes(prec, nc, f.Vh);
  if (f.norm) r.norm = f.norm + nblk * f.Vh;
  return r;
}

// zeroes the columns (and FP16 norms) that v covers; works on views
int vec_zero(Vec& v) {
  if (!v.ncol) return 0;
  const size_t nblk = (size_t)v.ncol * v.npar;
  if (launch_fill_zero(v.f.data, nblk * block_bytes(v.prec, v.nc, v.f.Vh), v.s) ||
      (v.f.norm && launch_fill_zero(v.f.norm, nblk * v.f.Vh * sizeof(float), v.s)))
    return fail(LQ_EDEVICE, "zero fill");
  return 0;
}

int vec_copy(Vec& dst, const Vec& src) {
  if (dst.ncol != src.ncol || dst.npar != src.npar || dst.nc != src.nc) return fail(LQ_EINVAL, "vec_copy: shape");
  return launch_convert(dst.f, dst.prec, src.f, src.prec, src.nc, src.ncol, src.npar, src.f.Vh, dst.s);
}

int vec_swap_cols(Vec& v, int a, int b) {
  if (a == b) return 0;
  if (a < 0 || b < 0 || a >= v.ncol || b >= v.ncol) return fail(LQ_EINVAL, "vec_swap_cols: column out of range");
  const size_t nblk = (size_t)v.npar;
  FieldRef fa = v.cols(a), fb = v.cols(b);
  if (launch_swap_bytes(fa.data, fb.data, nblk * block_bytes(v.prec, v.nc, v.f.Vh), v.s) ||
      (v.f.norm && launch_swap_bytes(fa.norm, fb.norm, nblk * v.f.Vh * sizeof(float), v.s)))
    return fail(LQ_EDEVICE, "column swap");
  return 0;
}

DBuf::DBuf(size_t bytes, hipStream_t st) : n(bytes), s(st) {
  if (bytes && hipMallocAsync(&p, bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
}
DBuf::~DBuf() {
  if (p) hipFreeAsync(p, s);
}

// ------------------------------------------------------------------ fields
int ensure_links(OpEnv& e, int prec) {
  lq_field* f = e.f;
  std::lock_guard<std::mutex> lk(f->mtx);
  const int pi = pidx(prec);
  const size_t esz = prec == 64 ? 16 : prec == 32 ? 8 : 4;
  if (f->type == 0) {
    const int rc = (e.recon && prec != 64) ? 1 : 0;
    if (f->links[pi][rc]) return 0;
    if (e.noalloc) return fail(LQ_EINVAL, "links of this precision are not resident (an earlier lq_apply or lq_solve "
                                          "at this precision packs them)");
    const int ne = rc ? 6 : 9;
    void* p = nullptr;
    if (hipMalloc(&p, esz * ne * 8 * (size_t)f->g.Vh) != hipSuccess) return fail(LQ_ENOMEM, "link allocation");
    int r = launch_pack_links(f->g, f->aos, p, prec, ne, 0, 1.0, e.s);
    // complete before publishing: other streams (server engines, API calls) may use the field next
    if (r || hipStreamSynchronize(e.s) != hipSuccess) return fail(LQ_EDEVICE, "pack links");
    f->links[pi][rc] = p;
    return 0;
  }
  if (f->fat[pi]) return 0;
  if (e.noalloc) return fail(LQ_EINVAL, "links of this precision are not resident (an earlier lq_apply or lq_solve "
                                        "at this precision packs them)");
  double sf = 1.0, sl = 1.0;
  if (prec == 16) {
    const int64_t n = 2 * (int64_t)f->g.Vh * 4 * 18;
    sf = 0.5 * link_maxabs(f->aos, n, e.s);
    sl = 0.5 * link_maxabs(f->aos2, n, e.s);
    if (!(sf > 0)) sf = 1.0;
    if (!(sl > 0)) sl = 1.0;
  }
  void *pf = nullptr, *pl = nullptr;
  const size_t bytes = esz * 9 * 8 * (size_t)f->g.Vh;
  if (hipMalloc(&pf, bytes) != hipSuccess || hipMalloc(&pl, bytes) != hipSuccess)
    return fail(LQ_ENOMEM, "HISQ link allocation");
  if (launch_pack_links(f->g, f->aos, pf, prec, 9, 1, sf, e.s) ||
      launch_pack_links(f->g, f->aos2, pl, prec, 9, 3, sl, e.s) || hipStreamSynchronize(e.s) != hipSuccess)
    return fail(LQ_EDEVICE, "pack HISQ links");
  f->fat[pi] = pf;
  f->lng[pi] = pl;
  f->sfat[pi] = (float)sf;
  f->slng[pi] = (float)sl;
  return 0;
}

int ensure_clover(OpEnv& e, int prec) {
  if (prec == 16) return fail(LQ_ENOTSUP, "the clover term is stored in FP64 or FP32 only");
  int r = ensure_links(e, 64);
  if (r) return r;
  lq_field* f = e.f;
  std::lock_guard<std::mutex> lk(f->mtx);
  auto key = std::make_tuple(e.act.m, e.act.c_sw, e.act.mu);
  if (e.noalloc) {
    auto it = f->clover.find(key);
    if (it == f->clover.end() || !it->second.H[pidx(prec)])
      return fail(LQ_EINVAL, "the clover term of this action and precision is not resident (an earlier lq_apply or "
                             "lq_solve builds it)");
    return 0;
  }
  Clover& c = f->clover[key];
  const size_t nH = 2 * 2 * 18 * (size_t)f->g.Vh, nA = 2 * 2 * 36 * (size_t)f->g.Vh;  // T2 elements
  if (!c.H[0]) {
    if (hipMalloc(&c.H[0], nH * 16) != hipSuccess || hipMalloc(&c.Ainv[0], nA * 16) != hipSuccess)
      return fail(LQ_ENOMEM, "clover allocation");
    if (launch_clover_build(f->g, f->links[0][0], e.act.c_sw, e.act.m, e.act.mu, c.H[0], c.Ainv[0], e.s) ||
        hipStreamSynchronize(e.s) != hipSuccess)
      return fail(LQ_EDEVICE, "clover build");
  }
  if (prec == 32 && !c.H[1]) {
    if (hipMalloc(&c.H[1], nH * 8) != hipSuccess || hipMalloc(&c.Ainv[1], nA * 8) != hipSuccess)
      return fail(LQ_ENOMEM, "clover allocation");
    if (launch_clover_convert(c.H[0], c.H[1], (int64_t)nH, e.s) ||
        launch_clover_convert(c.Ainv[0], c.Ainv[1], (int64_t)nA, e.s) || hipStreamSynchronize(e.s) != hipSuccess)
      return fail(LQ_EDEVICE, "clover convert");
  }
  return 0;
}

const Clover* get_clover(OpEnv& e) {
  std::lock_guard<std::mutex> lk(e.f->mtx);  // map nodes are stable; lookups race with inserts only
  auto it = e.f->clover.find(std::make_tuple(e.act.m, e.act.c_sw, e.act.mu));
  return it == e.f->clover.end() ? nullptr : &it->second;
}

static void* links_for(OpEnv& e, int prec) { return e.f->links[pidx(prec)][(e.recon && prec != 64) ? 1 : 0]; }

// per-site compulsory bytes: links read once, every field operand once
static double wilson_bytes(int prec, int recon, int n_fields, int ncol, int clov_mats) {
  const double r = prec == 64 ? 8 : prec == 32 ? 4 : 2;
  const double link = 8 * (recon && prec != 64 ? 12 : 18) * r;
  const double spin = 24 * r + (prec == 16 ? 4 : 0);
  const double clov = clov_mats * 72 * (prec == 64 ? 8 : 4);
  return link + clov + (double)ncol * n_fields * spin;
}

// ------------------------------------------------------------------ autotuner
// Launch shapes (columns per thread NR, traversal slab depth) are chosen per
// kernel key by timing every candidate on the real operands into a scratch
// output (all candidates compute each column with identical arithmetic).
// LQ_TUNE=0 disables tuning (NR=1, lexicographic order); LQ_TUNE_CACHE=<file>
// persists choices.
static bool tune_enabled() {
  const char* v = getenv("LQ_TUNE");
  return !(v && v[0] == '0');
}

static void tune_load(lq_ctx* c) {
  if (c->tune_loaded) return;
  c->tune_loaded = true;
  const char* path = getenv("LQ_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[256];
  Shape sh{};
  while (fscanf(f, "%255s %d %d %d %d", key, &sh.nr, &sh.slab, &sh.tpb, &sh.xcd) == 5) c->tune[key] = sh;
  fclose(f);
}

static void tune_save(lq_ctx* c) {
  const char* path = getenv("LQ_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (auto& kv : c->tune)
    fprintf(f, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.nr, kv.second.slab, kv.second.tpb, kv.second.xcd);
  fclose(f);
}

// Traversal orders worth trying for a lattice: lexicographic, z slabs of
// 1-8 planes, and the (y, z, t) blocks of whole x rows with the least surface
// per site among those of 1.5k-6k sites (about what one XCD has in flight).
static std::vector<int> slab_candidates(const Geom& g) {
  std::vector<int> v{0};
  for (int bz : {1, 2, 4, 8})
    if (g.L[2] % bz == 0 && bz < g.L[2]) v.push_back(bz);
  struct Blk {
    double surf;
    int code;
  };
  std::vector<Blk> blocks;
  for (int by : {2, 3, 4, 6, 8, 12, 16})
    for (int bz : {2, 3, 4, 6, 8, 12, 16})
      for (int bt : {2, 4, 8, 16, 32}) {
        if (g.L[1] % by || g.L[2] % bz || g.L[3] % bt) continue;
        if (by == g.L[1] && bt == g.L[3]) continue;  // a z slab, listed above
        const long sites = (long)g.Lxh * by * bz * bt;
        if (sites < 1536 || sites > 6144) continue;
        blocks.push_back({1.0 / by + 1.0 / bz + 1.0 / bt, traversal_code(by, bz, bt)});
      }
  std::sort(blocks.begin(), blocks.end(), [](const Blk& a, const Blk& b) { return a.surf < b.surf; });
  for (size_t k = 0; k < blocks.size() && k < 6; ++k) v.push_back(blocks[k].code);
  return v;
}

template <typename Args>
static void apply_shape(Args& A, const Shape& sh) {
  A.nr = sh.nr;
  A.slab = sh.slab;
  A.tpb = sh.tpb;
  A.xcd = sh.xcd;
}

template <typename Args, typename LaunchFn>
static int tuned(lq_ctx* c, const std::string& key, Args& A, size_t out_bytes, int prec,
                 const std::vector<int>& nrs, hipStream_t s, LaunchFn launch, bool may_tune = true) {
  const std::vector<int> slabs = slab_candidates(A.g);
  Shape choice{1, 0, 0, 1};
  if (const char* f = getenv("LQ_TUNE_FORCE")) {
    // testing hook: force "nr,order[,tpb,xcd]" (nr where it is a candidate, any valid traversal order)
    int nr = 1, bz = 0, tpb = 0, xcd = 1;
    if (sscanf(f, "%d,%d,%d,%d", &nr, &bz, &tpb, &xcd) >= 2) {
      Shape sh{std::find(nrs.begin(), nrs.end(), nr) != nrs.end() ? nr : 1, traversal_valid(A.g, bz) ? bz : 0,
               (tpb == 1 || tpb == 2 || tpb == 4 || tpb == 8) ? tpb : 0, xcd ? 1 : 0};
      apply_shape(A, sh);
      return launch(A, s);
    }
  }
  bool need = false;
  {
    std::lock_guard<std::mutex> lk(c->mtx);
    tune_load(c);
    auto it = c->tune.find(key);
    if (it != c->tune.end()) choice = it->second;
    else if (!may_tune) choice = Shape{1, 0, 0, 1};  // untuned default, not recorded
    else if (!tune_enabled()) c->tune[key] = choice;
    else need = true;
  }
  if (need) {
    // scratch output: main part rounded to 256 bytes, FP16 norms after it
    const size_t main_bytes = (out_bytes + 255) / 256 * 256;
    const size_t norm_bytes = prec == 16 ? out_bytes / 3 + 256 : 0;  // >= sites * 4 (FP16 site_bytes >= 12)
    DBuf scratch(main_bytes + norm_bytes, s);
    Args B = A;
    B.out.data = scratch.p;
    if (prec == 16) B.out.norm = (float*)((char*)scratch.p + main_bytes);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best = 1e30f;
    auto trial = [&](const Shape& sh) {
      apply_shape(B, sh);
      // one untimed launch (also sizes the timing: long launches are timed once)
      hipEventRecord(e0, s);
      if (!scratch.p || launch(B, s)) {
        (void)hipGetLastError();
        return;
      }
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float first = 0.f;
      hipEventElapsedTime(&first, e0, e1);
      const int reps = first > 2.0f ? 1 : 3;
      hipEventRecord(e0, s);
      for (int k = 0; k < reps; ++k) launch(B, s);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best) {
        best = ms;
        choice = sh;
      }
    };
    // coordinate search: columns per thread, traversal order, columns per
    // thread again at that order, then tiles per workgroup x block order, each
    // around the best shape so far
    for (int nr : nrs) trial(Shape{nr, 0, 0, 1});
    const Shape s0 = choice;
    for (int bz : slabs)
      if (bz != 0) trial(Shape{s0.nr, bz, 0, 1});
    const Shape sb = choice;
    for (int nr : nrs)
      if (nr != sb.nr) trial(Shape{nr, sb.slab, 0, 1});
    const Shape s1 = choice;
    for (int tpb : {0, 1, 2, 4, 8})
      for (int xcd : {1, 0})
        if (!(tpb == 0 && xcd == 1)) trial(Shape{s1.nr, s1.slab, tpb, xcd});
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(c->mtx);
    c->tune[key] = choice;
    tune_save(c);
  }
  apply_shape(A, choice);
  return launch(A, s);
}

// Column-count class of a tuning key: widths between two classes share the
// shape tuned for the first launch in the class (solvers that drop converged
// columns launch at many widths).
static int col_bucket(int n) {
  int b = 1;
  for (int c : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256}) {
    b = c;
    if (c >= n) break;
  }
  return n > b ? n : b;
}

// bytes of the value part of an output with ncol columns x npar parities
// (FP16: site_bytes >= 12, so a third of it covers the 4-byte site norms)
static size_t tune_out_bytes(int prec, int nc, int ncol, int npar, int Vh) {
  return (size_t)ncol * npar * Vh * (size_t)site_bytes(prec, nc);
}

static std::vector<int> nr_candidates(int prec, int ncol, bool blocked) {
  std::vector<int> v{1};
  if (!blocked) return v;
  for (int nr : {2, 3, 4, 6})
    if (nr <= ncol && !(prec == 64 && nr > 4)) v.push_back(nr);
  return v;
}

static int run_wilson(OpEnv& e, WilsonArgs& A, int n_fields, int clov_mats, int flops_extra) {
  A.g = e.f->g;
  if (A.ncol <= 0) return 0;  // nothing to compute
  A.recon = (e.recon && A.prec != 64) ? 1 : 0;
  if (!A.links) return fail(LQ_EDEVICE, "links not packed");
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  static const char* epi_names[] = {"hop", "xpay", "xpay_g5", "clovinv", "xmy", "site", "cheb", "xmyt", "clovinv_x"};
  char name[48];
  snprintf(name, sizeof(name), "wilson%d_%s", A.prec, epi_names[A.epi]);
  char key[160];
  snprintf(key, sizeof(key), "%s_r%d_d%d_n%d_v%d_p%d", name, A.recon, A.dag, col_bucket(A.ncol), A.g.Vh, A.par_out);
  const bool blocked = !A.dag && (A.epi == EPI_CLOVINV || A.epi == EPI_XMY_CLOVINV || A.epi == EPI_XPAY ||
                                  A.epi == EPI_XPAY_G5 || A.epi == EPI_CHEB || A.epi == EPI_XMY_RTS ||
                                  A.epi == EPI_SITE || A.epi == EPI_CLOVINV_XPAY);
  const int out_npar = A.out.npar;
  // timed under the kernel's name and under name_n<columns> (solvers that drop
  // converged columns launch the same kernel at several widths)
  char name_n[64];
  snprintf(name_n, sizeof(name_n), "%s_n%d", name, A.ncol);
  const double launch_bytes = (double)nsite * wilson_bytes(A.prec, A.recon, n_fields, A.ncol, clov_mats);
  Prof p(e.noalloc ? nullptr : e.ctx, name, e.s, launch_bytes);
  Prof pn(e.noalloc ? nullptr : e.ctx, name_n, e.s, launch_bytes);
  int r = tuned(e.ctx, key, A, tune_out_bytes(A.prec, 12, A.ncol, out_npar, A.g.Vh), A.prec,
                nr_candidates(A.prec, A.ncol, blocked), e.s,
                [](const WilsonArgs& B, hipStream_t st) { return launch_wilson(B, st); }, !e.noalloc);
  if (r) return fail(r == -1 ? LQ_ENOTSUP : LQ_EDEVICE, "wilson stencil launch");
  e.n_apply += A.par_out == 2 ? 2 : 1;
  e.flops += (double)nsite * A.ncol * (1320.0 + flops_extra);
  e.bytes += launch_bytes;
  return 0;
}

// ------------------------------------------------------------------ Wilson type
int wilson_D(OpEnv& e, int prec, Vec& out, const Vec& in, bool dag) {
  int r = ensure_links(e, prec);
  if (r) return r;
  WilsonArgs A{};
  A.prec = prec;
  A.dag = dag;
  A.par_out = 2;
  A.ncol = in.ncol;
  A.links = links_for(e, prec);
  A.in = in.f;
  A.out = out.f;
  A.x = in.f;
  A.k_hop = -0.5;
  if (e.act.kind == LQ_TM_CLOVER) {
    r = ensure_clover(e, prec);
    if (r) return r;
    A.epi = EPI_SITE;
    A.clov = get_clover(e)->H[pidx(prec)];
    A.mu_tw = dag ? -e.act.mu : e.act.mu;
    return run_wilson(e, A, 3, 1, 504);
  }
  A.epi = EPI_XPAY;
  A.a = 4.0 + e.act.m;
  return run_wilson(e, A, 3, 0, 48);
}

int wilson_hop(OpEnv& e, int prec, Vec& out, const Vec& in) {
  int r = ensure_links(e, prec);
  if (r) return r;
  WilsonArgs A{};
  A.prec = prec;
  A.par_out = 2;
  A.ncol = in.ncol;
  A.links = links_for(e, prec);
  A.in = in.f;
  A.out = out.f;
  A.k_hop = -0.5;
  A.epi = EPI_HOP;
  return run_wilson(e, A, 2, 0, 0);
}

int tm_site(OpEnv& e, int prec, Vec& out, const Vec& in, bool inverse) {
  int r = ensure_clover(e, prec);
  if (r) return r;
  const Clover* c = get_clover(e);
  Prof p(e.ctx, "site", e.s);
  r = launch_site(e.f->g, prec, c->H[pidx(prec)], c->Ainv[pidx(prec)], e.act.mu, inverse, in.f, out.f,
                  in.npar == 2 ? 2 : in.par0, in.ncol, e.s);
  return r ? fail(LQ_EDEVICE, "site kernel") : 0;
}

int tm_schur(OpEnv& e, int prec, Vec& out_e, const Vec& in_e, Vec& tmp_o, int red_mode, double* red) {
  int r = ensure_links(e, prec);
  if (!r) r = ensure_clover(e, prec);
  if (r) return r;
  const Clover* c = get_clover(e);
  WilsonArgs A{};
  A.prec = prec;
  A.ncol = in_e.ncol;
  A.links = links_for(e, prec);
  A.k_hop = -0.5;
  A.clov_inv = c->Ainv[pidx(prec)];
  A.in = in_e.f;
  A.out = tmp_o.f;
  A.par_out = 1;
  A.epi = EPI_CLOVINV;
  r = run_wilson(e, A, 2, 2, 576);
  if (r) return r;
  A.in = tmp_o.f;
  A.out = out_e.f;
  A.x = in_e.f;
  A.par_out = 0;
  A.epi = EPI_XMY_CLOVINV;
  if (red_mode == 2 && red) {
    A.epi = EPI_XMY_RTS;
    A.red = red;
    return run_wilson(e, A, 3, 2, 672);
  }
  return run_wilson(e, A, 3, 2, 600);
}

int tm_schur_source(OpEnv& e, Vec& bhat_e, const Vec& b) {
  const int prec = b.prec;
  int r = ensure_links(e, prec);
  if (!r) r = ensure_clover(e, prec);
  if (r) return r;
  const Clover* c = get_clover(e);
  const Geom& g = e.f->g;
  Vec t_o = make_vec(g, prec, 12, b.ncol, 1, 1, e.s);
  if (!t_o.ok()) return fail(LQ_ENOMEM, "schur source buffers");
  // t_o = A_oo^-1 b_o, then b_hat_e = A_ee^-1 (b_e + 1/2 hop(t_o)) in one stencil
  if (launch_site(g, prec, c->H[pidx(prec)], c->Ainv[pidx(prec)], e.act.mu, true, b.f, t_o.f, 1, b.ncol, e.s))
    return fail(LQ_EDEVICE, "site");
  WilsonArgs A{};
  A.prec = prec;
  A.ncol = b.ncol;
  A.links = links_for(e, prec);
  A.in = t_o.f;
  A.out = bhat_e.f;
  A.x = b.f;
  A.clov_inv = c->Ainv[pidx(prec)];
  A.k_hop = 0.5;
  A.par_out = 0;
  A.epi = EPI_CLOVINV_XPAY;
  return run_wilson(e, A, 3, 2, 600);
}

int tm_schur_reconstruct(OpEnv& e, Vec& x, const Vec& x_e, const Vec& b) {
  const int prec = x.prec;
  int r = ensure_links(e, prec);
  if (!r) r = ensure_clover(e, prec);
  if (r) return r;
  const Clover* c = get_clover(e);
  WilsonArgs A{};
  A.prec = prec;
  A.ncol = b.ncol;
  A.links = links_for(e, prec);
  // x_e into the even half of x (hop scaled by zero)
  A.in = x_e.f;
  A.out = x.f;
  A.x = x_e.f;
  A.a = 1.0;
  A.k_hop = 0.0;
  A.par_out = 0;
  A.epi = EPI_XPAY;
  r = run_wilson(e, A, 2, 0, 0);
  if (r) return r;
  // x_o = A_oo^-1 (b_o - D_oe x_e) = A_oo^-1 (b_o + 1/2 hop(x_e)) in one stencil
  A.out = x.f;
  A.x = b.f;
  A.clov_inv = c->Ainv[pidx(prec)];
  A.k_hop = 0.5;
  A.par_out = 1;
  A.epi = EPI_CLOVINV_XPAY;
  return run_wilson(e, A, 3, 2, 600);
}

// ------------------------------------------------------------------ overlap
int hw_apply(OpEnv& e, int prec, Vec& out, const Vec& in) {
  int r = ensure_links(e, prec);
  if (r) return r;
  WilsonArgs A{};
  A.prec = prec;
  A.par_out = 2;
  A.ncol = in.ncol;
  A.links = links_for(e, prec);
  A.in = in.f;
  A.out = out.f;
  A.x = in.f;
  A.a = 4.0 - e.act.rho;
  A.k_hop = -0.5;
  A.epi = EPI_XPAY_G5;
  return run_wilson(e, A, 3, 0, 48);
}

// Lanczos steps for the H_W^2 interval of the Chebyshev approximation
#ifndef LQ_HW_LANCZOS
#define LQ_HW_LANCZOS 300
#endif

// The Chebyshev interval [a, b] must hold the spectrum of H_W^2 (sec. 2.3).
// The Lanczos spectrum of H_W(rho) is measured once per field and rho.  With
// no interval given, a = 0.9 (theta_min - r_min) and b = 1.1 (theta_max + r_max)
// (certified Ritz bounds with a margin); a given interval is refused
// (LQ_EINVAL) when a Ritz value lies outside it, since Ritz values lie inside
// the spectrum.
int overlap_prepare(OpEnv& e) {
  if (!e.cheb.empty()) return 0;
  if (e.act.cheb_N < 1) return fail(LQ_EINVAL, "overlap: cheb_N must be >= 1");
  HwSpectrum sp{};
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(e.f->mtx);
    auto it = e.f->hw_spec.find(e.act.rho);
    if (it != e.f->hw_spec.end()) {
      sp = it->second;
      have = true;
    }
  }
  if (!have) {
    int r = hw_spectrum(e.ctx, &e.act, e.f, LQ_HW_LANCZOS, &sp, e.s);
    if (r) return r;
    std::lock_guard<std::mutex> lk(e.f->mtx);
    e.f->hw_spec[e.act.rho] = sp;
  }
  double a = e.act.cheb_a, b = e.act.cheb_b;
  const int nl = e.act.n_lowmodes;
  if (nl > 0) {
    // low modes treated exactly: the polynomial must hold the rest of the spectrum
    const EigSet* es = find_eigs(e.f, LQ_EIG_HW, e.act.rho, 0);
    if (!es || es->n < nl + 1)
      return fail(LQ_EINVAL, "overlap: n_lowmodes needs at least n_lowmodes + 1 resident H_W modes (lq_eigs)");
    if (!(a > 0 && b > a)) {
      a = 0.9 * es->vals[nl] * es->vals[nl];
      b = 1.1 * (sp.theta_max + sp.r_max);
    } else if (sp.theta_max > b || a > es->vals[nl] * es->vals[nl]) {
      return fail(LQ_EINVAL, "overlap: the Chebyshev interval does not hold the spectrum outside the low modes");
    }
  } else if (a > 0 && b > a) {
    if (sp.theta_min < a || sp.theta_max > b)
      return fail(LQ_EINVAL, "overlap: the Chebyshev interval [" + std::to_string(a) + ", " + std::to_string(b) +
                                 "] does not hold the spectrum of H_W^2 (Ritz values " +
                                 std::to_string(sp.theta_min) + ", " + std::to_string(sp.theta_max) + ")");
  } else {
    a = 0.9 * (sp.theta_min - sp.r_min);
    b = 1.1 * (sp.theta_max + sp.r_max);
  }
  e.a = a;
  e.b = b;
  e.cheb.assign(e.act.cheb_N + 1, 0.0);
  if (e.act.cheb_c) std::memcpy(e.cheb.data(), e.act.cheb_c, sizeof(double) * (e.act.cheb_N + 1));
  else cheb_coeffs(a, b, e.act.cheb_N, e.cheb.data());
  return 0;
}

static int sign_poly(OpEnv& e, int prec, Vec& out, const Vec& in);

// eps(H_W) v; with n_lowmodes > 0 the low modes of H_W enter exactly:
// eps v = sum_i sign(lambda_i) u_i <u_i, v> + P eps_N(H_W) P v, with the
// projections and the low-mode part in FP64 and the polynomial in `prec`
int sign_apply(OpEnv& e, int prec, Vec& out, const Vec& in) {
  int r = overlap_prepare(e);
  if (r) return r;
  const int nl = e.act.n_lowmodes;
  if (nl <= 0) return sign_poly(e, prec, out, in);
  const Geom& g = e.f->g;
  const EigSet* es = find_eigs(e.f, LQ_EIG_HW, e.act.rho, 0);
  if (!es || es->n < nl) return fail(LQ_EINVAL, "overlap: low modes not resident");
  Vec v64 = make_vec(g, 64, 12, in.ncol, 2, 0, e.s), o64 = make_vec(g, 64, 12, in.ncol, 2, 0, e.s);
  DBuf coef(sizeof(double) * 2 * nl * std::max(in.ncol, 1), e.s), junk(sizeof(double) * 2 * nl * std::max(in.ncol, 1), e.s);
  if (!v64.ok() || !o64.ok() || !coef.p || !junk.p) return fail(LQ_ENOMEM, "projection buffers");
  if ((r = vec_copy(v64, in))) return r;
  if ((r = project_out(e.ctx, g, e.s, *es, nl, v64, coef.p))) return r;
  if (prec == 64) {
    if ((r = sign_poly(e, 64, o64, v64))) return r;
  } else {
    Vec vl = make_vec(g, prec, 12, in.ncol, 2, 0, e.s), ol = make_vec(g, prec, 12, in.ncol, 2, 0, e.s);
    if (!vl.ok() || !ol.ok()) return fail(LQ_ENOMEM, "projection buffers");
    if ((r = vec_copy(vl, v64)) || (r = sign_poly(e, prec, ol, vl)) || (r = vec_copy(o64, ol))) return r;
  }
  if ((r = project_out(e.ctx, g, e.s, *es, nl, o64, junk.p))) return r;
  std::vector<double> w((size_t)nl * in.ncol);
  for (int col = 0; col < in.ncol; ++col)
    for (int i = 0; i < nl; ++i) w[(size_t)col * nl + i] = es->vals[i] >= 0 ? 1.0 : -1.0;
  if ((r = add_modes(e.ctx, g, e.s, *es, nl, w, o64, coef.p))) return r;
  return vec_copy(out, o64);
}

// eps_N(H_W) v by Clenshaw's recursion (no projection)
static int sign_poly(OpEnv& e, int prec, Vec& out, const Vec& in) {
  int r = ensure_links(e, prec);
  if (r) return r;
  const Geom& g = e.f->g;
  const int N = (int)e.cheb.size() - 1;
  const double a = e.a, b = e.b;
  Vec bk1 = make_vec(g, prec, 12, in.ncol, 2, 0, e.s);
  Vec bk2 = make_vec(g, prec, 12, in.ncol, 2, 0, e.s);
  Vec w = make_vec(g, prec, 12, in.ncol, 2, 0, e.s);
  if (!bk1.ok() || !bk2.ok() || !w.ok()) return fail(LQ_ENOMEM, "sign buffers");
  Blas bl;
  if ((r = blas_prepare(e.ctx, bl, g, 2, in.ncol, e.s))) return r;
  // b_N = c_N v ; b_{N+1} = 0
  BlasArgs A{};
  {
    BlasArgs B{};
    B.prec = prec; B.nc = 12; B.ncol = in.ncol; B.npar = 2; B.Vh = g.Vh; B.op = OP_LC_G5;
    B.f[0] = in.f; B.f[1] = in.f; B.f[2] = bk1.f; B.imm[0] = e.cheb[N]; B.gridx = bl.gridx;
    BlasProf p(e.ctx, B, e.s);
    if (launch_blas(B, e.s)) return fail(LQ_EDEVICE, "blas");
  }
  if ((r = vec_zero(bk2))) return fail(LQ_EDEVICE, "zero");
  WilsonArgs W{};
  W.prec = prec;
  W.par_out = 2;
  W.ncol = in.ncol;
  W.links = links_for(e, prec);
  W.a = 4.0 - e.act.rho;
  W.k_hop = -0.5;
  W.epi = EPI_CHEB;
  W.v = in.f;
  for (int k = N - 1; k >= 0; --k) {
    if ((r = hw_apply(e, prec, w, bk1))) return r;
    W.in = w.f;
    W.x = w.f;
    W.b1 = bk1.f;
    W.b2 = bk2.f;
    W.out = bk2.f;
    W.ck = e.cheb[k];
    if (k > 0) {
      W.s1 = 4.0 / (b - a);
      W.s2 = -2.0 * (a + b) / (b - a);
    } else {
      W.s1 = 2.0 / (b - a);
      W.s2 = -(a + b) / (b - a);
    }
    if ((r = run_wilson(e, W, 6, 0, 96))) return r;
    std::swap(bk1, bk2);  // bk1 = b_k, bk2 = b_{k+1}
  }
  (void)A;
  // bk1 now holds y = sum_k c_k T_k(Z) v
  return hw_apply(e, prec, out, bk1);
}

int cheb_filter(OpEnv& e, Vec& out, const Vec& in, double lo, double hi, int d) {
  int r = ensure_links(e, 64);
  if (r) return r;
  const Geom& g = e.f->g;
  // T_0 = v, T_1 = Z v, T_{j+1} = 2 Z T_j - T_{j-1}: each step one H_W and one
  // stencil with the Clenshaw epilogue (c_k = 0)
  Vec t0 = make_vec(g, 64, 12, in.ncol, 2, 0, e.s), t1 = make_vec(g, 64, 12, in.ncol, 2, 0, e.s),
      w = make_vec(g, 64, 12, in.ncol, 2, 0, e.s);
  if (!t0.ok() || !t1.ok() || !w.ok()) return fail(LQ_ENOMEM, "filter buffers");
  if ((r = vec_copy(t0, in)) || (r = vec_zero(t1))) return r;
  WilsonArgs W{};
  W.prec = 64;
  W.par_out = 2;
  W.ncol = in.ncol;
  W.links = links_for(e, 64);
  W.a = 4.0 - e.act.rho;
  W.k_hop = -0.5;
  W.epi = EPI_CHEB;
  W.ck = 0.0;
  for (int j = 0; j < d; ++j) {
    // t1 <- s1 H(H t0) + s2 t0 - t1 (j = 0: Z v with the halved factors, t1 = 0)
    if ((r = hw_apply(e, 64, w, t0))) return r;
    W.in = w.f;
    W.x = w.f;
    W.v = t0.f;
    W.b1 = t0.f;
    W.b2 = t1.f;
    W.out = t1.f;
    W.s1 = (j == 0 ? 2.0 : 4.0) / (hi - lo);
    W.s2 = (j == 0 ? -1.0 : -2.0) * (lo + hi) / (hi - lo);
    if ((r = run_wilson(e, W, 6, 0, 96))) return r;
    std::swap(t0, t1);  // t0 = T_{j+1}, t1 = T_j
  }
  return vec_copy(out, t0);
}

int overlap_D(OpEnv& e, int prec, Vec& out, const Vec& in, bool dag) {
  const Geom& g = e.f->g;
  Blas bl;
  int r = blas_prepare(e.ctx, bl, g, 2, in.ncol, e.s);
  if (r) return r;
  const double rho = e.act.rho, m = e.act.m;
  Vec ein = make_vec(g, prec, 12, in.ncol, 2, 0, e.s);
  Vec eps = make_vec(g, prec, 12, in.ncol, 2, 0, e.s);
  if (!ein.ok() || !eps.ok()) return fail(LQ_ENOMEM, "overlap buffers");
  const Vec* src = &in;
  if (dag) {
    if ((r = bl.op(OP_G5, const_cast<Vec*>(&in), &ein))) return r;
    src = &ein;
  }
  if ((r = sign_apply(e, prec, eps, *src))) return r;
  BlasArgs B{};
  B.prec = prec; B.nc = 12; B.ncol = in.ncol; B.npar = 2; B.Vh = g.Vh; B.op = OP_LC_G5;
  B.f[0] = src->f; B.f[1] = eps.f; B.f[2] = dag ? ein.f : out.f; B.gridx = bl.gridx;
  B.imm[0] = rho + 0.5 * m;
  B.imm[2] = rho - 0.5 * m;
  {
    BlasProf p(e.ctx, B, e.s);
    if (launch_blas(B, e.s)) return fail(LQ_EDEVICE, "blas");
  }
  if (dag) return bl.op(OP_G5, &ein, &out);
  return 0;
}

// ------------------------------------------------------------------ staggered
static int run_stag(OpEnv& e, StagArgs& A, int n_fields) {
  A.g = e.f->g;
  if (A.ncol <= 0) return 0;  // nothing to compute (the kernel reads column ncol - 1)
  const int pi = pidx(A.prec);
  A.fat = e.f->fat[pi];
  A.lng = e.f->lng[pi];
  A.sfat = e.f->sfat[pi];
  A.slong = e.f->slng[pi];
  const int nsite = A.par_out == 2 ? 2 * A.g.Vh : A.g.Vh;
  char name[48];
  snprintf(name, sizeof(name), "stag%d_%s", A.prec, A.epi == SEPI_HOP ? "hop" : A.epi == SEPI_XPAY ? "xpay" : "xpayd");
  char key[160];
  snprintf(key, sizeof(key), "%s_n%d_v%d_p%d", name, col_bucket(A.ncol), A.g.Vh, A.par_out);
  std::vector<int> nrs{1};
  for (int nr : {2, 3, 4, 6, 8})
    if (nr <= A.ncol && !(A.prec == 64 && nr > 4)) nrs.push_back(nr);
  // timed under the kernel's name and under name_n<columns> (solvers that drop
  // converged columns launch the same kernel at several widths)
  char name_n[64];
  snprintf(name_n, sizeof(name_n), "%s_n%d", name, A.ncol);
  const double rb = A.prec == 64 ? 8 : A.prec == 32 ? 4 : 2;
  const double launch_bytes =
      (double)nsite * (16 * 18 * rb + (double)A.ncol * n_fields * (6 * rb + (A.prec == 16 ? 4 : 0)));
  Prof p(e.noalloc ? nullptr : e.ctx, name, e.s, launch_bytes);
  Prof pn(e.noalloc ? nullptr : e.ctx, name_n, e.s, launch_bytes);
  if (tuned(e.ctx, key, A, tune_out_bytes(A.prec, 3, A.ncol, A.out.npar, A.g.Vh), A.prec, nrs, e.s,
            [](const StagArgs& B, hipStream_t st) { return launch_stag(B, st); }, !e.noalloc))
    return fail(LQ_EDEVICE, "staggered stencil launch");
  e.n_apply += A.par_out == 2 ? 2 : 1;
  e.flops += (double)nsite * A.ncol * 1146.0;
  e.bytes += launch_bytes;
  return 0;
}

int stag_D(OpEnv& e, int prec, Vec& out, const Vec& in, bool dag, const double* acol_dev) {
  int r = ensure_links(e, prec);
  if (r) return r;
  StagArgs A{};
  A.prec = prec;
  A.epi = SEPI_XPAY;
  A.par_out = 2;
  A.ncol = in.ncol;
  A.in = in.f;
  A.out = out.f;
  A.x = in.f;
  A.a = e.act.m;
  A.acol = acol_dev;
  A.k_hop = dag ? -1.0 : 1.0;
  return run_stag(e, A, 3);
}

int stag_hop(OpEnv& e, int prec, Vec& out, const Vec& in) {
  int r = ensure_links(e, prec);
  if (r) return r;
  StagArgs A{};
  A.prec = prec;
  A.epi = SEPI_HOP;
  A.par_out = 2;
  A.ncol = in.ncol;
  A.in = in.f;
  A.out = out.f;
  A.k_hop = 1.0;
  return run_stag(e, A, 2);
}

int stag_normal_even(OpEnv& e, int prec, Vec& out_e, const Vec& in_e, Vec& tmp_o, const double* acol_dev, double a,
                     double* red) {
  int r = ensure_links(e, prec);
  if (r) return r;
  StagArgs A{};
  A.prec = prec;
  A.ncol = in_e.ncol;
  A.epi = SEPI_HOP;
  A.par_out = 1;
  A.in = in_e.f;
  A.out = tmp_o.f;
  A.k_hop = 1.0;
  if ((r = run_stag(e, A, 2))) return r;
  A.epi = SEPI_XPAY;
  A.par_out = 0;
  A.in = tmp_o.f;
  A.out = out_e.f;
  A.x = in_e.f;
  A.acol = acol_dev;
  A.a = a;
  A.k_hop = -1.0;
  if (red) {
    A.epi = SEPI_XPAY_DOT;
    A.red = red;
  }
  return run_stag(e, A, 3);
}

// ------------------------------------------------------------------ BLAS helper
int blas_prepare(lq_ctx* c, Blas& b, const Geom& g, int npar, int ncol, hipStream_t s) {
  b.ctx = c;
  b.s = s;
  b.gridx = blas_gridx((int64_t)npar * g.Vh);
  const size_t need = (size_t)std::max(ncol, 1) * b.gridx * 4 * sizeof(double);
  b.part = DBuf(need, s);
  if (!b.part.p) return fail(LQ_ENOMEM, "reduction buffer");
  b.partial = b.part.as<double>();
  return 0;
}

int Blas::op(int opc, Vec* f0, Vec* f1, Vec* f2, Vec* f3, Vec* f4, const double* st, int c0, int c1) {
  BlasArgs A{};
  A.prec = f0->prec;
  A.nc = f0->nc;
  A.ncol = f0->ncol;
  A.npar = f0->npar;
  A.Vh = f0->f.Vh;
  A.op = opc;
  Vec* fs[5] = {f0, f1, f2, f3, f4};
  for (int k = 0; k < 5; ++k) {
    if (!fs[k]) continue;
    if (fs[k]->prec != A.prec || fs[k]->npar != A.npar || fs[k]->ncol < A.ncol)
      return fail(LQ_EINVAL, "blas: operand shape/precision mismatch");
    A.f[k] = fs[k]->f;
  }
  A.st = st;
  A.c0 = c0;
  A.c1 = c1;
  A.partial = partial;
  A.gridx = gridx;
  BlasProf p(ctx, A, s);
  return launch_blas(A, s) ? fail(LQ_EDEVICE, "blas launch") : 0;
}

int Blas::opi(int opc, Vec* f0, Vec* f1, Vec* f2, double c0re, double c0im, double c1re, double c1im) {
  BlasArgs A{};
  A.prec = f0->prec;
  A.nc = f0->nc;
  A.ncol = f0->ncol;
  A.npar = f0->npar;
  A.Vh = f0->f.Vh;
  A.op = opc;
  A.f[0] = f0->f;
  if (f1) A.f[1] = f1->f;
  if (f2) A.f[2] = f2->f;
  A.imm[0] = c0re;
  A.imm[1] = c0im;
  A.imm[2] = c1re;
  A.imm[3] = c1im;
  A.partial = partial;
  A.gridx = gridx;
  BlasProf p(ctx, A, s);
  return launch_blas(A, s) ? fail(LQ_EDEVICE, "blas launch") : 0;
}

int Blas::plc(Vec* f0, Vec* f1, Vec* f2, const double* pcol) {
  BlasArgs A{};
  A.prec = f0->prec;
  A.nc = f0->nc;
  A.ncol = f0->ncol;
  A.npar = f0->npar;
  A.Vh = f0->f.Vh;
  A.op = OP_PLC;
  Vec* fs[3] = {f0, f1, f2};
  for (int k = 0; k < 3; ++k) {
    if (fs[k]->prec != A.prec || fs[k]->npar != A.npar || fs[k]->ncol < A.ncol || fs[k]->nc != 12)
      return fail(LQ_EINVAL, "blas: operand shape/precision mismatch");
    A.f[k] = fs[k]->f;
  }
  A.pcol = pcol;
  A.partial = partial;
  A.gridx = gridx;
  BlasProf p(ctx, A, s);
  return launch_blas(A, s) ? fail(LQ_EDEVICE, "blas launch") : 0;
}

// ------------------------------------------------------------------ Chebyshev
void cheb_coeffs(double a, double b, int N, double* c) {
  // interpolation of y^{-1/2} at the N+1 Chebyshev nodes of [a, b]; c_0 halved
  const double pi = 3.14159265358979323846;
  std::vector<double> f(N + 1), th(N + 1);
  for (int j = 0; j <= N; ++j) {
    th[j] = pi * (j + 0.5) / (N + 1);
    const double y = 0.5 * (b - a) * std::cos(th[j]) + 0.5 * (b + a);
    f[j] = 1.0 / std::sqrt(y);
  }
  for (int k = 0; k <= N; ++k) {
    double s = 0.0;
    for (int j = 0; j <= N; ++j) s += std::cos(k * th[j]) * f[j];
    c[k] = 2.0 * s / (N + 1);
  }
  c[0] *= 0.5;
}

}  // namespace lq
