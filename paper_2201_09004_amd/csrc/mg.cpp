// Host side of the two-level aggregation multigrid (sec. 2.1, Table 2):
// aggregate maps, the basis and the Galerkin coarse operator, the transfer and
// coarse operators on solver vectors, and the host-array entry point.
//
// The coarse operator is assembled by probing the fine operator.  Aggregates
// are coloured by the parities of their coarse coordinates (16 classes);
// for a class c and a coarse component k the probe is the prolongation of the
// unit vector e_k on every aggregate of class c.  D applied to it reaches only
// those aggregates and their nearest neighbours, whose classes differ from c
// in one bit, and the neighbour in -mu and the one in +mu land on opposite
// faces of an aggregate at least two sites deep.  So one FP64 application of D
// per (class, component) gives column k of the self term of every class-c
// aggregate and of the two mu-links of every aggregate next to one: 16 x 2 nv
// applications in all, batched by columns.
#include <algorithm>
#include <cstring>
#include <vector>

#include "lq_internal.h"
#include "lq_kernels.h"

namespace lq {

namespace {

int upload_ints(int** dst, const std::vector<int>& v, hipStream_t s) {
  if (hipMalloc((void**)dst, v.size() * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return fail(LQ_ENOMEM, "multigrid maps");
  }
  if (hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LQ_EDEVICE, "multigrid maps");
  return 0;
}

void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

}  // namespace

void mg_release(MgHier* h) {
  if (!h) return;
  for (void* p : {(void*)h->fine, (void*)h->nbr, (void*)h->face, (void*)h->cpar, (void*)h->cmap, (void*)h->csite,
                  h->Q64, h->Q32, h->Dc64, h->Dc32, h->Ahat64, h->Ahat32})
    if (p) hipFree(p);
  delete h;
}

bool mg_matches(const MgHier* h, const lq_action* act) {
  return h && act && h->kind == act->kind && h->m == act->m && h->mu == (act->kind == LQ_TM_CLOVER ? act->mu : 0.0) &&
         h->csw == (act->kind == LQ_TM_CLOVER ? act->c_sw : 0.0);
}

int mg_init_maps(MgHier& h, const Geom& g, const int block[4], int nv) {
  h.nv = nv;
  h.K = 2 * nv / 12;
  h.B = 1;
  h.Vc = 1;
  for (int mu = 0; mu < 4; ++mu) {
    h.block[mu] = block[mu];
    h.Lc[mu] = g.L[mu] / block[mu];
    h.B *= block[mu];
    h.Vc *= h.Lc[mu];
  }
  std::vector<int> fine((size_t)h.Vc * h.B), face((size_t)h.Vc * h.B), nbr((size_t)h.Vc * 8), cpar(h.Vc);
  std::vector<int> cmap(h.Vc), csite(h.Vc);
  const int* Lc = h.Lc;
  int ncb[2] = {0, 0};
  for (int Y = 0; Y < h.Vc; ++Y) {
    int yc[4];
    int r = Y;
    for (int mu = 0; mu < 4; ++mu) {
      yc[mu] = r % Lc[mu];
      r /= Lc[mu];
    }
    cpar[Y] = (yc[0] & 1) | (yc[1] & 1) << 1 | (yc[2] & 1) << 2 | (yc[3] & 1) << 3;
    const int cp = (yc[0] + yc[1] + yc[2] + yc[3]) & 1;
    const int cb = ncb[cp]++;
    cmap[Y] = cb | cp << 30;
    csite[cp * (h.Vc / 2) + cb] = Y;
    for (int mu = 0; mu < 4; ++mu)
      for (int sgn = 0; sgn < 2; ++sgn) {
        int zc[4] = {yc[0], yc[1], yc[2], yc[3]};
        zc[mu] = (zc[mu] + (sgn == 0 ? 1 : Lc[mu] - 1)) % Lc[mu];
        nbr[(size_t)Y * 8 + 2 * mu + sgn] = zc[0] + Lc[0] * (zc[1] + Lc[1] * (zc[2] + Lc[2] * zc[3]));
      }
    for (int b = 0; b < h.B; ++b) {
      int bc[4], x[4];
      int q = b;
      for (int mu = 0; mu < 4; ++mu) {
        bc[mu] = q % block[mu];
        q /= block[mu];
        x[mu] = yc[mu] * block[mu] + bc[mu];
      }
      const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
      const int cb = (x[0] >> 1) + g.Lxh * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
      fine[(size_t)Y * h.B + b] = cb | par << 30;
      int fb = 0;
      for (int mu = 0; mu < 4; ++mu) {
        if (bc[mu] == 0) fb |= 1 << (2 * mu);
        if (bc[mu] == block[mu] - 1) fb |= 1 << (2 * mu + 1);
      }
      face[(size_t)Y * h.B + b] = fb;
    }
  }
  hipStream_t s = nullptr;
  int e = upload_ints(&h.fine, fine, s);
  if (!e) e = upload_ints(&h.face, face, s);
  if (!e) e = upload_ints(&h.nbr, nbr, s);
  if (!e) e = upload_ints(&h.cpar, cpar, s);
  if (!e) e = upload_ints(&h.cmap, cmap, s);
  if (!e) e = upload_ints(&h.csite, csite, s);
  if (e) return e;
  if (ncb[0] != h.Vc / 2 || ncb[1] != h.Vc / 2) return fail(LQ_EINVAL, "multigrid: odd coarse lattice");
  h.cmap_h = cmap;
  h.gc = g;
  h.gc.Vh = h.K * h.Vc / 2;
  return 0;
}

int mg_build(OpEnv& e, MgHier& h, Vec& vecs) {
  hipStream_t s = e.s;
  const MgGeom m = h.geom();
  const int n2 = 2 * h.nv;
  const size_t nq = (size_t)h.Vc * h.B * 2 * h.nv * 6;  // complex entries of Q
  const size_t nd = (size_t)h.Vc * 9 * n2 * n2;          // complex entries of Dc
  h.Q64 = dev_alloc(nq * 16);
  h.Q32 = dev_alloc(nq * 8);
  h.Dc64 = dev_alloc(nd * 16);
  h.Dc32 = dev_alloc(nd * 8);
  if (!h.Q64 || !h.Q32 || !h.Dc64 || !h.Dc32) return fail(LQ_ENOMEM, "multigrid basis and coarse operator");
  DBuf bad(sizeof(int), s);
  if (!bad.p) return fail(LQ_ENOMEM, "multigrid");
  if (launch_fill_zero(bad.p, sizeof(int), s) || launch_mg_gather(m, vecs.f, h.Q64, s) ||
      launch_mg_orth(m, h.Q64, bad.as<int>(), s) || launch_mg_narrow(h.Q64, h.Q32, (int64_t)nq, s) ||
      launch_fill_zero(h.Dc64, nd * 16, s))
    return fail(LQ_EDEVICE, "multigrid basis");
  int nbad = 0;
  if (hipMemcpyAsync(&nbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LQ_EDEVICE, "multigrid basis");
  if (nbad) return fail(LQ_ENUMERIC, "multigrid: a near-null vector vanishes on an aggregate");
  // probing, 12 coarse components at a time
  const int nb = std::min(12, n2);
  Vec pf = make_vec(e.f->g, 64, 12, nb, 2, 0, s);
  Vec df = make_vec(e.f->g, 64, 12, nb, 2, 0, s);
  if (!pf.ok() || !df.ok()) return fail(LQ_ENOMEM, "multigrid probes");
  for (int cls = 0; cls < 16; ++cls)
    for (int k0 = 0; k0 < n2; k0 += nb) {
      const int w = std::min(nb, n2 - k0);
      Vec pfw = view(pf, 0, w), dfw = view(df, 0, w);
      if (launch_mg_probe_fine(m, h.Q64, pfw.f, w, k0, cls, s)) return fail(LQ_EDEVICE, "multigrid probe");
      int r = wilson_D(e, 64, dfw, pfw, false);
      if (r) return r;
      if (launch_mg_probe_restrict(m, h.Q64, dfw.f, w, k0, cls, h.Dc64, s)) return fail(LQ_EDEVICE, "multigrid probe");
    }
  if (launch_mg_narrow(h.Dc64, h.Dc32, (int64_t)nd, s)) return fail(LQ_EDEVICE, "multigrid coarse operator");
  // the even-odd preconditioned coarse operator: A^{-1} and A^{-1} Dc[d]
  h.Ahat64 = dev_alloc(nd * 16);
  h.Ahat32 = dev_alloc(nd * 8);
  DBuf work((size_t)h.Vc * n2 * 2 * n2 * 16, s);
  if (!h.Ahat64 || !h.Ahat32 || !work.p) return fail(LQ_ENOMEM, "multigrid coarse operator");
  if (launch_fill_zero(bad.p, sizeof(int), s) || launch_mg_site_inverse(m, h.Dc64, h.Ahat64, work.p, bad.as<int>(), s) ||
      launch_mg_site_mul(m, h.Dc64, h.Ahat64, s) || launch_mg_narrow(h.Ahat64, h.Ahat32, (int64_t)nd, s))
    return fail(LQ_EDEVICE, "multigrid coarse operator");
  if (hipMemcpyAsync(&nbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LQ_EDEVICE, "multigrid setup");
  if (nbad) return fail(LQ_ENUMERIC, "multigrid: singular self block of the coarse operator");
  return 0;
}

int mg_restrict(OpEnv& e, const MgHier& h, const Vec& fine, Vec& coarse) {
  Prof p(e.ctx, "mg_restrict", e.s, (double)h.Vc * h.B * 12 * fine.ncol * (fine.prec == 64 ? 16 : 8) +
                                        (double)h.Vc * h.B * 2 * h.nv * 6 * (fine.prec == 64 ? 16 : 8));
  const void* Q = fine.prec == 64 ? h.Q64 : h.Q32;
  return launch_mg_restrict(h.geom(), fine.prec, Q, fine.f, coarse.prec, coarse.f, fine.ncol, e.s)
             ? fail(LQ_EDEVICE, "multigrid restriction")
             : 0;
}

int mg_prolong(OpEnv& e, const MgHier& h, const Vec& coarse, Vec& fine) {
  Prof p(e.ctx, "mg_prolong", e.s, (double)h.Vc * h.B * 12 * fine.ncol * (fine.prec == 64 ? 16 : 8) +
                                       (double)h.Vc * h.B * 2 * h.nv * 6 * (fine.prec == 64 ? 16 : 8));
  const void* Q = fine.prec == 64 ? h.Q64 : h.Q32;
  return launch_mg_prolong(h.geom(), coarse.prec, coarse.f, fine.prec, Q, fine.f, coarse.ncol, e.s)
             ? fail(LQ_EDEVICE, "multigrid prolongation")
             : 0;
}

int mg_coarse_op(OpEnv& e, const MgHier& h, Vec& out, const Vec& in) {
  const int n2 = 2 * h.nv;
  const double bytes = (double)h.Vc * 9 * n2 * n2 * (in.prec == 64 ? 16 : 8) +
                       2.0 * h.Vc * n2 * in.ncol * (in.prec == 64 ? 16 : 8);
  Prof p(e.ctx, in.prec == 64 ? "mg_coarse64" : "mg_coarse32", e.s, bytes);
  e.n_apply += 1;
  e.bytes += bytes;
  return launch_mg_stencil(h.geom(), in.prec, in.prec == 64 ? h.Dc64 : h.Dc32, 0, 9, in.f, out.f, in.f, 0.0, 1.0, 2,
                           in.ncol, e.s)
             ? fail(LQ_EDEVICE, "multigrid coarse operator")
             : 0;
}

namespace {
// one launch of the coarse stencil on half the aggregates, timed as mg_hop<P>
int hop_half(OpEnv& e, const MgHier& h, int prec, int d0, int nd, const Vec& in, Vec& out, const Vec& x, double a,
             double sgn, int par_out) {
  const int n2 = 2 * h.nv;
  const double bytes = (double)h.Vc / 2 * nd * n2 * n2 * (prec == 64 ? 16 : 8) +
                       (2.0 + (a != 0.0)) * h.Vc / 2 * n2 * in.ncol * (prec == 64 ? 16 : 8);
  Prof p(e.ctx, prec == 64 ? "mg_hop64" : "mg_hop32", e.s, bytes);
  e.bytes += bytes;
  return launch_mg_stencil(h.geom(), prec, prec == 64 ? h.Ahat64 : h.Ahat32, d0, nd, in.f, out.f, x.f, a, sgn, par_out,
                           in.ncol, e.s)
             ? fail(LQ_EDEVICE, "multigrid coarse stencil")
             : 0;
}
}  // namespace

int mg_schur_source(OpEnv& e, const MgHier& h, Vec& bhat_e, Vec& t_o, Vec& u_e, const Vec& b) {
  int r = hop_half(e, h, b.prec, 0, 1, b, t_o, b, 0.0, 1.0, 1);          // t_o = A_oo^-1 b_o
  if (!r) r = hop_half(e, h, b.prec, 1, 8, t_o, u_e, t_o, 0.0, 1.0, 0);  // u_e = A_ee^-1 D_eo t_o
  if (!r) r = hop_half(e, h, b.prec, 0, 1, b, bhat_e, u_e, -1.0, 1.0, 0);  // A_ee^-1 b_e - u_e
  return r;
}

int mg_schur_op(OpEnv& e, const MgHier& h, Vec& out_e, const Vec& in_e, Vec& tmp_o) {
  e.n_apply += 1;
  int r = hop_half(e, h, in_e.prec, 1, 8, in_e, tmp_o, in_e, 0.0, 1.0, 1);
  if (!r) r = hop_half(e, h, in_e.prec, 1, 8, tmp_o, out_e, in_e, 1.0, -1.0, 0);
  return r;
}

int mg_schur_reconstruct(OpEnv& e, const MgHier& h, Vec& x, const Vec& x_e, const Vec& t_o) {
  int r = hop_half(e, h, x.prec, 0, 0, x_e, x, x_e, 1.0, 1.0, 0);           // x_e into x
  if (!r) r = hop_half(e, h, x.prec, 1, 8, x_e, x, t_o, 1.0, -1.0, 1);      // x_o = t_o - A_oo^-1 D_oe x_e
  return r;
}

// ------------------------------------------------------------------ host arrays
namespace {

// coarse Vec (FP64) <-> host [n][Vc][2][nv] complex
int coarse_to_host(const MgHier& h, const Vec& v, double* out, hipStream_t s) {
  std::vector<double> raw(v.bytes / 8);
  if (hipMemcpyAsync(raw.data(), v.f.data, v.bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LQ_EDEVICE, "copy");
  const int n2 = 2 * h.nv;
  for (int col = 0; col < v.ncol; ++col)
    for (int Y = 0; Y < h.Vc; ++Y)
      for (int d = 0; d < n2; ++d) {
        const int cm = h.cmap_h[Y];
        const int64_t i = tix((int64_t)col * 2 + ((cm >> 30) & 1), d % 12, 12, (cm & 0x3fffffff) * h.K + d / 12,
                              h.gc.Vh);
        double* o = out + 2 * (((int64_t)col * h.Vc + Y) * n2 + d);
        o[0] = raw[2 * i];
        o[1] = raw[2 * i + 1];
      }
  return 0;
}

int coarse_from_host(const MgHier& h, Vec& v, const double* in, hipStream_t s) {
  std::vector<double> raw(v.bytes / 8, 0.0);
  const int n2 = 2 * h.nv;
  for (int col = 0; col < v.ncol; ++col)
    for (int Y = 0; Y < h.Vc; ++Y)
      for (int d = 0; d < n2; ++d) {
        const int cm = h.cmap_h[Y];
        const int64_t i = tix((int64_t)col * 2 + ((cm >> 30) & 1), d % 12, 12, (cm & 0x3fffffff) * h.K + d / 12,
                              h.gc.Vh);
        const double* x = in + 2 * (((int64_t)col * h.Vc + Y) * n2 + d);
        raw[2 * i] = x[0];
        raw[2 * i + 1] = x[1];
      }
  if (hipMemcpyAsync(v.f.data, raw.data(), v.bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LQ_EDEVICE, "copy");
  return 0;
}

}  // namespace

int mg_apply_host(lq_ctx* c, const lq_action* act, lq_field* f, int op, int prec, int n, const double* in,
                  double* out, hipStream_t s) {
  MgHier* h = f->mg;
  if (!mg_matches(h, act)) return fail(LQ_EINVAL, "no multigrid setup for this action on this field");
  if (prec != 64 && prec != 32) return fail(LQ_EINVAL, "prec_bits must be 64 or 32");
  if (op < LQ_MG_RESTRICT || op > LQ_MG_COARSE) return fail(LQ_EINVAL, "unknown multigrid operator");
  if (n <= 0) return 0;
  const Geom& g = f->g;
  OpEnv env{c, f, *act, s};
  const size_t fine_doubles = (size_t)n * 2 * g.Vh * 24;
  const size_t coarse_doubles = (size_t)n * h->Vc * 2 * h->nv * 2;
  Vec c64 = make_vec(h->gc, 64, 12, n, 2, 0, s);
  Vec clo = make_vec(h->gc, prec, 12, n, 2, 0, s);
  Vec f64 = make_vec(g, 64, 12, n, 2, 0, s);
  Vec flo = make_vec(g, prec, 12, n, 2, 0, s);
  DBuf aos(sizeof(double) * std::max(fine_doubles, coarse_doubles), s);
  if (!c64.ok() || !clo.ok() || !f64.ok() || !flo.ok() || !aos.p) return fail(LQ_ENOMEM, "multigrid buffers");
  int e = 0;
  if (op == LQ_MG_RESTRICT) {
    if (hipMemcpyAsync(aos.p, in, fine_doubles * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(LQ_EDEVICE, "copy");
    if (launch_pack_field(g, aos.as<double>(), n, 12, f64.f, 64, 2, s)) return fail(LQ_EDEVICE, "pack");
    if ((e = vec_copy(flo, f64)) || (e = mg_restrict(env, *h, flo, c64))) return e;
    return coarse_to_host(*h, c64, out, s);
  }
  if ((e = coarse_from_host(*h, c64, in, s))) return e;
  if (op == LQ_MG_PROLONG) {
    if ((e = mg_prolong(env, *h, c64, flo)) || (e = vec_copy(f64, flo))) return e;
    if (launch_unpack_field(g, f64.f, 64, n, 12, aos.as<double>(), 2, s)) return fail(LQ_EDEVICE, "unpack");
    if (hipMemcpyAsync(out, aos.p, fine_doubles * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LQ_EDEVICE, "copy");
    return 0;
  }
  Vec olo = make_vec(h->gc, prec, 12, n, 2, 0, s);
  if (!olo.ok()) return fail(LQ_ENOMEM, "multigrid buffers");
  if ((e = vec_copy(clo, c64)) || (e = mg_coarse_op(env, *h, olo, clo)) || (e = vec_copy(c64, olo))) return e;
  return coarse_to_host(*h, c64, out, s);
}

}  // namespace lq
