/* liblq: lattice Dirac-operator solvers for AMD MI355X (gfx950).
 *
 * The calls follow the problem statement of arXiv:2201.09004 ("Performance
 * of the GPU inverters with Chroma+QUDA for various fermion actions"):
 * compute a propagator, i.e. solve D(U; m, omega, c_sw) x = b column by column
 * (12 spin-colour columns for Wilson-type actions, sec. 2.1 and Table 2;
 * 3 colour columns for staggered, sec. 2.2 and Table 3) to a stated
 * residual, for the twisted-mass clover (sec. 2.1, eqs. 1-3), HISQ staggered
 * (sec. 2.2, eq. 4) and overlap (sec. 2.3, eq. 5 and the sign-function form
 * that follows it) actions.
 *
 * Conventions (shared by every entry point):
 *   - extents L = {Lx, Ly, Lz, Lt}, all even (>= 4 for HISQ so that the
 *     three-hop Naik term does not alias); site s = x + Lx*(y + Ly*(z + Lz*t));
 *     mu = 0..3 is x, y, z, t; parity = (x+y+z+t) & 1, even = 0.
 *   - gauge links: [V][4][3][3] complex128 (re, im interleaved), U_mu(x)[row][col]
 *     the link from x to x + mu.  Space is periodic; with t_antiperiodic the
 *     library applies the fermion time-boundary sign itself.
 *   - Wilson-type fields: [n_rhs][V][4][3] complex128 (spin, colour), chiral
 *     gamma basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
 *     gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 *   - staggered fields: [n_rhs][V][3] complex128.  HISQ fat (one-hop) and long
 *     (three-hop) links are passed with smearing and Naik coefficients
 *     absorbed and WITHOUT staggered phases; the library applies the MILC
 *     phases eta_t = 1, eta_x = (-1)^t, eta_y = (-1)^(t+x), eta_z = (-1)^(t+x+y).
 *
 * Operators (kind and op codes below):
 *   D_W(m)  = (4+m) - 1/2 sum_mu [(1-g_mu) U_mu(x) d_{x+mu} + (1+g_mu) U^dag_mu(x-mu) d_{x-mu}]
 *             (eq. 2 read with the standard sign; eq. 2 as printed is -g5 D_W g5)
 *   TM-clover D = D_W(m) + C + i mu g5, C = -(c_sw/2) sum_{mu<nu} g_mu g_nu F_mu_nu
 *             (eq. 1 with omega = m + i mu on i g5, eq. 3 with the Luescher normalisation)
 *   HISQ     D = m + 1/2 sum_mu eta_mu [V d_{+mu} - V^dag d_{-mu} + W d_{+3mu} - W^dag d_{-3mu}]
 *   overlap  D(m) = (rho - m/2)(1 + g5 eps(H_W)) + m, H_W = g5 D_W(-rho),
 *             eps(H) v ~= H sum_{k=0}^{N} c_k T_k(Z) v, Z = (2 H^2 - (a+b))/(b-a),
 *             evaluated by Clenshaw's recursion (sec. 2.3, Fig. 2).
 *
 * Errors: every call returns lq_status (0 = LQ_OK, negative on error) and
 * never aborts; lq_last_error() gives a message for the calling thread.
 * Ownership: host pointers are borrowed for the duration of the call and
 * copied; lq_field handles belong to the library until lq_field_free; the
 * _dev variants borrow caller device memory (same canonical layouts, FP64)
 * and enqueue on the caller's HIP stream, returning after the work is
 * enqueued and the stats are final (they synchronise that stream).
 */
#ifndef LQ_H
#define LQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LQ_OK = 0,
  LQ_EINVAL = -1,     /* bad argument: odd extent, unknown kind/op, bad sizes, NULL pointer */
  LQ_ENOMEM = -2,     /* device allocation failed (or server budget exceeded) */
  LQ_EDEVICE = -3,    /* HIP runtime error */
  LQ_ENOCONV = -4,    /* maxiter reached; x holds the best iterate, stats are filled */
  LQ_EBREAKDOWN = -5, /* BiCGStab breakdown that a restart did not cure */
  LQ_ENUMERIC = -6,   /* NaN or Inf in a reduction */
  LQ_EBUSY = -7,      /* server: request not finished / queue full */
  LQ_ENOTSUP = -8     /* combination not supported (e.g. FP16 with clover) */
} lq_status;

typedef struct lq_ctx lq_ctx;
typedef struct lq_field lq_field;
typedef struct lq_server lq_server;

typedef struct {
  int32_t L[4];           /* Lx, Ly, Lz, Lt: all even; Lx Ly Lz Lt / 2 <= 2^31 / 64 (else LQ_EINVAL) */
  int32_t t_antiperiodic; /* 1: antiperiodic fermion time boundary (default) */
} lq_geom;

enum { LQ_WILSON = 0, LQ_TM_CLOVER = 1, LQ_HISQ = 2, LQ_OVERLAP = 3 };

typedef struct {
  int32_t kind;       /* LQ_WILSON, LQ_TM_CLOVER, LQ_HISQ, LQ_OVERLAP */
  double m;           /* Wilson/TM mass m of D_W(m) (Re omega); HISQ mass; overlap quark mass */
  double mu;          /* twisted mass (Im omega), TM only */
  double c_sw;        /* clover coefficient, TM only (0: no clover term) */
  double rho;         /* overlap: D_W(-rho) kernel, rho ~ 1.5 */
  int32_t cheb_N;     /* overlap: polynomial order in H^2 (2N+1 H_W products) */
  double cheb_a;      /* overlap: interval [a, b] holding the spectrum of H_W^2 (both 0: the */
  double cheb_b;      /*   library takes a = 0.9 lmin^2, b = 1.1 lmax^2 from lq_hw_bounds; a
                           given interval that excludes a Lanczos Ritz value of H_W^2 is
                           refused with LQ_EINVAL) */
  const double *cheb_c; /* overlap: N+1 coefficients (host), or NULL: the library
                           interpolates y^(-1/2) at the Chebyshev nodes of [a,b] */
  int32_t n_lowmodes; /* overlap: low modes of H_W treated exactly in the sign function
                         (sec. 2.3): eps v = sum_i sign(lambda_i) u_i <u_i, v> + P eps_N(H_W) P v,
                         P = 1 - sum_i u_i u_i^dag, over the n_lowmodes smallest |lambda| of the
                         field's resident modes (lq_eigs with LQ_EIG_HW, which must hold at least
                         n_lowmodes + 1; else LQ_EINVAL).  With no interval given, a = 0.9 times
                         the square of the next mode's eigenvalue.  0: no projection. */
} lq_action;

/* operator selector for lq_apply (the result is written for every site of
 * `out` that the operator defines; other sites are set to zero) */
enum {
  LQ_OP_D = 0,         /* full-lattice D of the action */
  LQ_OP_DDAG = 1,      /* D^dag */
  LQ_OP_HOP = 2,       /* hopping part: Wilson -1/2 sum(...), HISQ D - m */
  LQ_OP_SITE = 3,      /* TM: site term A = (4+m) + C + i mu g5 */
  LQ_OP_SITE_INV = 4,  /* TM: A^{-1} */
  LQ_OP_SCHUR = 5,     /* TM: M_hat = 1 - A_ee^-1 D_eo A_oo^-1 D_oe on even sites */
  LQ_OP_HW = 6,        /* overlap: H_W = g5 D_W(-rho) */
  LQ_OP_SIGN = 7,      /* overlap: eps_N(H_W) */
  LQ_OP_NORMAL_EVEN = 8 /* HISQ: M_e(m) = m^2 - D_eo D_oe on even sites */
};

typedef struct {
  double tol;              /* target relative true residual ||b - D x|| / ||b|| (FP64) */
  int32_t maxiter;         /* iteration cap of the main Krylov loop (0: 10000) */
  int32_t sloppy_bits;     /* 64, 32 or 16: storage of the inner iterations (HISQ
                              multi-shift with 16: the multi-shift stage runs in FP32
                              to 1e-8, the per-shift refinement in FP16) */
  double reliable_delta;   /* reliable update when ||r|| < delta * max ||r|| since the last one (0: 0.1) */
  int32_t n_shift;         /* HISQ / overlap multi-mass: number of masses (0 or 1: single mass = action.m) */
  const double *masses;    /* HISQ / overlap multi-mass: n_shift masses (host) */
  int32_t reconstruct_full;/* HISQ: 1 returns x_i = D(m_i)^dag y_i on all sites, 0 returns y_i on even sites */
  int32_t recon12;         /* 1: 12-real link reconstruction in sloppy FP32/FP16 Wilson stencils */
  int32_t use_initial_guess;/* 1: x holds the initial guess on input */
  int32_t fault_inject;    /* testing: 1 NaN in the first reduction, 2 allocation failure, 3 maxiter=1 */
  int32_t solver;          /* 0: default for the action, 1: CG on normal equations D^dag D (full lattice,
                              twisted clover and overlap), 2: twisted clover even-odd flexible GCR(8)
                              in FP64, each direction from a sloppy BiCGStab to 0.1 of the residual
                              (at most 50 iterations), restarted from the true residual; 3: flexible
                              GCR on the full lattice preconditioned by the two-level multigrid of
                              lq_mg_setup (Wilson and twisted clover; LQ_EINVAL without a setup for
                              the same action on this field) */
  int32_t deflate;         /* overlap (solver 0): use this many resident chiral-sector low modes per
                              chirality (lq_eigs with LQ_EIG_OVERLAP) for the initial guess of every
                              sector solve; 0: none */
} lq_params;

typedef struct {
  int32_t iters;           /* Krylov iterations of the main loop (max over columns) */
  int32_t reliable_updates;
  double true_rel_res;     /* max over columns (and shifts) of the FP64 relative true residual */
  double seconds;          /* wall time of the call */
  double gflops;           /* stencil flops / seconds / 1e9 (standard per-site counts) */
  double hbm_bytes;        /* compulsory HBM bytes of the stencil applications */
  int32_t status;
  int32_t n_apply;         /* stencil (half-)applications issued */
} lq_stats;

/* Context on one device.  `device` is the HIP device ordinal. */
lq_status lq_init(int device, lq_ctx **ctx);
lq_status lq_finalize(lq_ctx *ctx);
/* Message of the last failed call on this thread (static storage, valid until the next call). */
const char *lq_last_error(void);
/* Library version string. */
const char *lq_version(void);

/* Gauge field for Wilson-type actions.  U: host [V][4][3][3] complex128 (SU(3)
 * for the 12-real reconstruction).  The clover term is built on the device
 * from U when an action with c_sw != 0 first needs it (sec. 2.1: the clover
 * term and its twisted inverse are computed on the GPU). */
lq_status lq_gauge_load(lq_ctx *ctx, const lq_geom *geom, const double *U, lq_field **g);
lq_status lq_gauge_load_dev(lq_ctx *ctx, const lq_geom *geom, const double *U_dev, void *stream, lq_field **g);
/* HISQ fat (one-hop) and long (three-hop) links, host [V][4][3][3] complex128 each. */
lq_status lq_hisq_load(lq_ctx *ctx, const lq_geom *geom, const double *fat, const double *lng, lq_field **g);
lq_status lq_hisq_load_dev(lq_ctx *ctx, const lq_geom *geom, const double *fat_dev, const double *lng_dev,
                           void *stream, lq_field **g);
lq_status lq_field_free(lq_field *g);

/* Most columns one call may carry: n_rhs, times n_shift for several masses and
 * times 2 for the chirally projected overlap solve (its two chiral sectors).
 * The vector kernels put the columns on the second dimension of their launch
 * grid.  Larger calls are refused with LQ_EINVAL before any data is read. */
#define LQ_MAX_COLUMNS 65535

/* Apply one operator (op codes above) once to n_rhs columns, with field
 * storage of prec_bits = 64, 32 or 16 (FP16: values scaled by a per-site FP32
 * norm, FP32 accumulation), optionally OR-ed with LQ_PREC_RECON12 (FP32/FP16
 * Wilson-type links stored as two rows, the third rebuilt as conj(r0 x r1)).
 * in/out: canonical layouts, n_rhs columns (n_rhs = 0 is a no-op). */
#define LQ_PREC_RECON12 0x100
lq_status lq_apply(lq_ctx *ctx, const lq_action *act, const lq_field *g, int op, int prec_bits, int n_rhs,
                   const double *in, double *out);
lq_status lq_apply_dev(lq_ctx *ctx, const lq_action *act, const lq_field *g, int op, int prec_bits, int n_rhs,
                       const double *in_dev, double *out_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lq_apply_dev
 * with no device allocation, free or synchronisation.  Ops: LQ_OP_D,
 * LQ_OP_DDAG and LQ_OP_HOP for LQ_WILSON, LQ_TM_CLOVER and LQ_HISQ, LQ_OP_HW
 * and LQ_OP_HOP for LQ_OVERLAP (others: LQ_EINVAL).  The packed input and
 * output vectors live in a fixed 64 MiB device array of the library (one per
 * GPU, held until the process ends): 2 x n_rhs x V x 192 bytes (FP64
 * Wilson-type) must fit, else LQ_EINVAL with the sizes in the message.
 * Preconditions (else LQ_EINVAL): the field's links at this precision, and
 * for the twisted-clover D its clover term at this precision, are already on
 * the device (any earlier lq_apply or lq_solve with them puts them there).
 * Launch shapes are those an earlier call tuned, else the untuned default;
 * this call never tunes.  in_dev/out_dev: device arrays in the canonical
 * layout; the work is enqueued on `stream` and the call returns without
 * waiting: synchronise the stream before reading out_dev.  Every call on a
 * GPU uses that GPU's one array, so calls that overlap in time (other
 * streams, other threads or contexts on the same GPU) race: serialise them. */
lq_status lq_apply_noalloc(lq_ctx *ctx, const lq_action *act, const lq_field *g, int op, int prec_bits, int n_rhs,
                           const double *in_dev, double *out_dev, void *stream);

/* Solve D x = b for n_rhs columns to prm->tol relative true residual.
 *   LQ_WILSON:     CG on D^dag D (full lattice)
 *   LQ_TM_CLOVER:  even-odd (symmetric Schur) BiCGStab, sloppy storage + FP64 reliable updates
 *   LQ_HISQ:       multi-shift CG on M_e(m_i) = m_i^2 - D_eo D_oe (even sites), then a
 *                  per-shift mixed-precision CG refinement; x is [n_shift][n_rhs][V][3]
 *   LQ_OVERLAP:    chirally projected normal equations (sec. 2.3): on a source of chirality
 *                  s, D(m)^dag D(m) = (1 - m^2/(4 rho^2)) 2 rho^2 (1 + s P_s eps P_s) + m^2
 *                  needs one sign function per CG iteration; each source is split into
 *                  its chiral halves (a spin-colour point source has one), the sector
 *                  system is solved by CG with sloppy storage of the sign function and
 *                  FP64 reliable updates, x = D(m)^dag z, and the FP64 residual of the
 *                  full D(m) is corrected by further sector solves until it meets tol.
 *                  Several masses (n_shift, masses in (0, 2 rho)) share one multi-shift
 *                  CG (the masses are shifts of the same sector operator), then each is
 *                  refined; x is [n_shift][n_rhs][V][4][3].  solver = 1: plain CG on
 *                  D(m)^dag D(m) (two sign functions per iteration), one mass.
 * x: on input the initial guess if prm->use_initial_guess (one mass), on output the solution.
 * stats may be NULL. */
lq_status lq_solve(lq_ctx *ctx, const lq_action *act, const lq_field *g, const lq_params *prm, int n_rhs,
                   const double *b, double *x, lq_stats *stats);
lq_status lq_solve_dev(lq_ctx *ctx, const lq_action *act, const lq_field *g, const lq_params *prm, int n_rhs,
                       const double *b_dev, double *x_dev, lq_stats *stats, void *stream);

/* Interval [lmin, lmax] of |eigenvalues| of H_W = g5 D_W(-rho) (sec. 2.3: the
 * Chebyshev interval must hold the spectrum).  `iters` FP64 Lanczos steps on H_W^2
 * from a fixed random start give the extreme Ritz values theta and, from the Ritz
 * vectors, the FP64 residual norms r = |H_W^2 y - theta y|; the result is
 * lmin^2 = theta_min - r_min, lmax^2 = theta_max + r_max.  LQ_EINVAL when the
 * smallest Ritz pair has not converged (r_min >= theta_min / 2) or iters < 2. */
lq_status lq_hw_bounds(lq_ctx *ctx, const lq_action *act, const lq_field *g, int iters, double *lmin,
                       double *lmax);
/* Low modes (sec. 2.3), computed on the device and kept resident with the field
 * (replacing an earlier set of the same kind and rho) until lq_field_free:
 *   LQ_EIG_HW       the nev eigenpairs of H_W = g5 D_W(-rho) with the smallest |lambda|
 *                   (for lq_action.n_lowmodes); evals[nev] ascending in |lambda|.  Lanczos with
 *                   implicit restarts (shifted QR steps on the tridiagonal Hessenberg matrix) on
 *                   the Chebyshev polynomial T_d(Z(H_W^2)) that maps [filter_cut, b] onto [-1, 1]
 *                   (filter_degree d, 0: 24; filter_cut 0: 4 times the smallest eigenvalue of
 *                   H_W^2), then a Rayleigh-Ritz step with H_W.  LQ_EINVAL if a found mode lies
 *                   above the cut (raise filter_cut).
 *   LQ_EIG_OVERLAP  the nev smallest eigenpairs of the chirally projected D(0)^dag D(0) =
 *                   2 rho^2 (1 + s P_s eps P_s) in each chirality s = +1, -1 (for
 *                   lq_params.deflate), with the action's sign function (FP64; FP32 when
 *                   tol >= 1e-6, enough for a deflation guess); evals[2 nev]: s = +1
 *                   then s = -1, each ascending.
 * tol: residual target |A u - lambda u| relative to the operator norm (0: 1e-10);
 * max_restarts (0: 200).  stats: iters = restarts, n_apply = operator applications,
 * true_rel_res = largest residual.  LQ_ENOCONV: the modes are stored, some residual is
 * above tol. */
enum { LQ_EIG_HW = 0, LQ_EIG_OVERLAP = 1 };
lq_status lq_eigs(lq_ctx *ctx, const lq_action *act, const lq_field *g, int which, int nev, double tol,
                  int max_restarts, int filter_degree, double filter_cut, double *evals, lq_stats *stats);

/* Coefficients c_0..c_N of the Chebyshev interpolant of y^(-1/2) on [a, b] (host, FP64). */
lq_status lq_cheb_coeffs(double a, double b, int N, double *c);

/* ---- Multigrid (sec. 2.1, Table 2: the multigrid inverter and its reusable
 * subspace setup) ------------------------------------------------------------
 * Two-level aggregation multigrid for LQ_TM_CLOVER (the Wilson operator is the
 * case c_sw = mu = 0).  The lattice is cut into aggregates of block[0..3] sites
 * (coarse lattice L / block, x fastest).  n_vec near-null vectors are split by
 * chirality on every aggregate and orthonormalised there (Gram-Schmidt in vector
 * order), which gives the prolongator P; restriction is P^dag and the coarse
 * operator is the Galerkin product D_c = P^dag D P, a nearest-neighbour stencil
 * of (2 n_vec)^2 blocks.  The setup is kept with the field (one hierarchy per
 * field, replaced by the next setup, freed with the field) and used by lq_solve
 * with solver = 3: flexible GCR(gcr_kmax) on D x = b, its cycles in FP32 closed
 * by FP64 updates (lq_params.maxiter counts its steps, default 1000; three
 * cycles that cut the worst residual by less than 10% end the solve with
 * LQ_ENOCONV), each direction from one V-cycle in FP32: restrict the residual,
 * solve the even-odd preconditioned coarse system by BiCGStab to coarse_tol (at
 * most coarse_maxiter iterations), prolong, then nu_post minimal-residual steps
 * on the even-odd preconditioned fine system; with nu_pre > 0 the cycle first
 * takes nu_pre such steps on the residual it is given and restricts the
 * residual they leave.
 * Coarse vectors (lq_mg_apply): host [n_rhs][Vc][2][n_vec] complex, index 0 of
 * the chirality axis for gamma5 = +1 (spins 0, 1 of the chiral basis). */
typedef struct {
  int32_t block[4];        /* aggregate extents (x, y, z, t): each >= 2; L / block even and >= 2 */
  int32_t n_vec;           /* near-null vectors: 6, 12, 18, 24 or 30 (0: 30) */
  int32_t setup_passes;    /* inverse-iteration passes from random vectors (0: 2) */
  int32_t setup_maxiter;   /* even-odd BiCGStab iterations per pass at most (0: 200) */
  int32_t coarse_maxiter;  /* V-cycle: coarse BiCGStab iterations at most (0: 100) */
  double setup_tol;        /* relative residual of every setup solve (0: 1e-4) */
  double coarse_tol;       /* V-cycle: coarse relative residual (0: 0.1) */
  uint64_t seed;           /* random start vectors (splitmix64 of seed and element index) */
  const double *null_vecs; /* optional host [n_vec][V][4][3]: the near-null vectors themselves, no passes */
  int32_t nu_post;         /* minimal-residual smoothing steps on the fine level (0: 4) */
  int32_t gcr_kmax;        /* outer flexible GCR restart length (0: 8) */
  int32_t nu_pre;          /* minimal-residual steps before the coarse correction (0: none) */
  int32_t reserved;        /* must be 0 */
} lq_mg_params;

/* Computes and stores the hierarchy.  stats: iters = setup BiCGStab iterations,
 * seconds = setup time.  A setup replaces the field's previous hierarchy: it must
 * not run while a solve with solver = 3 on the same field is in progress.  LQ_EINVAL: action other than Wilson / twisted clover,
 * block or n_vec out of range; LQ_ENUMERIC: a vector vanishes on an aggregate. */
lq_status lq_mg_setup(lq_ctx *ctx, const lq_action *act, const lq_field *g, const lq_mg_params *mp,
                      lq_stats *stats);

/* The transfer and coarse operators of the stored hierarchy on host arrays (FP64
 * in and out; prec_bits 64 or 32 selects the basis and coarse-operator copy):
 *   LQ_MG_RESTRICT  in fine [n][V][4][3] -> out coarse [n][Vc][2][n_vec]
 *   LQ_MG_PROLONG   in coarse -> out fine
 *   LQ_MG_COARSE    in coarse -> out D_c in
 * LQ_EINVAL without a hierarchy for this action. */
enum { LQ_MG_RESTRICT = 0, LQ_MG_PROLONG = 1, LQ_MG_COARSE = 2 };
lq_status lq_mg_apply(lq_ctx *ctx, const lq_action *act, const lq_field *g, int op, int prec_bits, int n_rhs,
                      const double *in, double *out);

/* HBM calibration: a plain copy kernel (one 16-byte chunk per lane) moves
 * `bytes` between two device buffers the library allocates and frees;
 * after one untimed launch, `reps` launches are timed with HIP events and
 * *gbs = 2 * bytes / (average launch time) / 1e9 (read + write).  The
 * measured achievable bandwidth is the denominator reported beside the
 * 8 TB/s specification.  LQ_ENOMEM if the buffers cannot be allocated. */
lq_status lq_copy_bandwidth(lq_ctx *ctx, size_t bytes, int reps, double *gbs);

/* Kernel timing with HIP events on the stream each kernel is launched on.
 * enable=1 clears and starts recording; lq_profile_get returns, for kernel
 * family `name` ("wilson", "stag", "blas", ...), the launch count and the
 * average duration in milliseconds. */
lq_status lq_profile(lq_ctx *ctx, int enable);
lq_status lq_profile_get(lq_ctx *ctx, const char *name, int64_t *count, double *avg_ms);
/* Algorithmic bytes (every operand read once, every output written once) of
 * the launches timed under `name` since profiling was enabled.  Names: the
 * stencil kernels as above (wilson32_clovinv, stag16_xpayd, ... and their
 * _n<columns> forms), "blas<prec>_<op>" (axpy, cg, xpay, dot, bicg_xr, ...),
 * "ms<prec>_xr" and "ms<prec>_p" (multi-shift vector kernels) and "blas" for
 * all vector kernels together. */
lq_status lq_profile_bytes(lq_ctx *ctx, const char *name, double *bytes);

/* Serving: continuous batching of propagator solves (the 12 spin-colour
 * columns of sec. 2.1, the colour columns of sec. 2.2) on resident gauge
 * fields.  A worker thread keeps one engine per (field, action, tol, sloppy
 * precision, recon, reliable_delta); an engine holds up to max_cols columns
 * (1..256) and advances all of them by one Krylov iteration per step, on its
 * own stream, concurrently with the other engines.  Columns join at
 * iteration boundaries when a slot is free and leave as soon as their FP64
 * true residual meets tol.  A new engine is created only if its estimated
 * HBM footprint fits hbm_budget (0: 80% of the free device memory at
 * creation); idle engines are evicted least-recently-used first.  Requests
 * are admitted in arrival order; one that does not fit yet waits without
 * holding back later ones that do, and one whose engine alone exceeds the
 * budget ends with LQ_ENOMEM.  Fields must outlive the server (destroy the
 * server before lq_field_free).
 *   Supported: LQ_TM_CLOVER (even-odd BiCGStab, sloppy 32 or 64, x = full
 *   solution of D x = b) and LQ_HISQ with one mass m > 0 (mixed CG on
 *   M_e = m^2 - D_eo D_oe, x = even-site solution, odd sites 0; as lq_solve
 *   with reconstruct_full = 0).  Other kinds: LQ_ENOTSUP.
 * b and x: host arrays [n_rhs][V][spin][colour] complex (as lq_solve), owned
 * by the caller and left untouched (b) / not read (x) until the request is
 * done; stats (may be NULL) is filled when it is done (iters = max over its
 * columns, seconds = latency from submit).  n_rhs must be <= max_cols.
 * lq_wait blocks until done and returns the request's status (LQ_OK,
 * LQ_ENOCONV, or the error that ended it); lq_poll sets *done without
 * blocking.  Tickets stay valid until lq_server_destroy, which finishes the
 * queued and running requests first.  lq_server_stats: median and 99th
 * percentile latency (seconds) of finished requests and columns finished per
 * second since the first submit. */
lq_status lq_server_create(lq_ctx *ctx, size_t hbm_budget, int max_cols, lq_server **srv);
lq_status lq_server_destroy(lq_server *srv);
lq_status lq_submit(lq_server *srv, const lq_action *act, const lq_field *g, const lq_params *prm, int n_rhs,
                    const double *b, double *x, lq_stats *stats, uint64_t *ticket);
lq_status lq_poll(lq_server *srv, uint64_t ticket, int *done);
lq_status lq_wait(lq_server *srv, uint64_t ticket);
lq_status lq_server_stats(lq_server *srv, double *p50_s, double *p99_s, double *solves_per_s);

#ifdef __cplusplus
}
#endif

#endif /* LQ_H */
