"""GPU parity at the benchmark sizes, in the launch shapes the benchmark uses.

At 24^3 x 64 (twisted clover, overlap kernel) and 32^3 x 96 (HISQ) the oracle
is evaluated at sampled sites only (oracle.sampled, pinned against the
whole-lattice oracle on small lattices), except for the solvers, whose FP64
true residual is computed with the whole-lattice oracle operator.  Inputs are
the benchmark's: links exp(i 0.2 H) seed 1001 and the Table 1 parameters;
12 Gaussian columns for operator checks, 12 point sources for the solves.

The sampled sites are 16 random ones plus forced ones: every time slice next
to the antiperiodic boundary (t = 0, 1, Lt-2, Lt-1), where the boundary sign
and the wrap of the three-hop Naik term act, the first and the last 64-site
tile of the checkerboard layout, and the far corner of each slice.
Tolerances: relative L2 over the sampled outputs 1e-6 (FP32 storage) and 3e-3
(FP16 storage with per-site norms), as for the small lattices, and a per-site
maximum relative error of 1e-5 (FP32) and 1e-2 (FP16); 1e-10 relative true
residual for the solutions.
"""
import numpy as np
import pytest

import synth
from oracle import sampled as SM
from oracle import wilson as W
from paper_2201_09004_amd import lq as L

pytestmark = pytest.mark.gpu

LAT = (24, 24, 24, 64)
M, CSW, MU = -0.0695, 1.0509, 0.01
NS = 16  # sampled sites per check


SITE_TOL = {32: 1e-5, 16: 1e-2}


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def site_max_rel(got, want):
    """max over columns and sites of |got - want| / |want| at one site (all spin-colour components)."""
    ax = tuple(range(2, got.ndim))
    return float((np.sqrt((np.abs(got - want) ** 2).sum(axis=ax)) / np.sqrt((np.abs(want) ** 2).sum(axis=ax))).max())


def forced_sites(L, parity=None):
    """Sites (t, z, y, x) that every sampled check includes: the four time
    slices at the antiperiodic boundary, the first and last 64-site tiles of
    the checkerboard order (cb = x/2 + Lx/2 (y + Ly (z + Lz t))), and the far
    corner; with `parity`, x is moved by one where needed."""
    Lx, Ly, Lz, Lt = L
    raw = []
    for t in (0, 1, Lt - 2, Lt - 1):
        raw += [(t, 0, 0, 0), (t, Lz - 1, Ly - 1, Lx - 1), (t, Lz // 2, 1, Lx - 2)]
    # the first 64 and the last 64 checkerboard sites span 128 / (Lx/2) rows of y
    rows = max(1, 128 // Lx)
    for k in range(rows):
        raw += [(0, 0, k % Ly, 1), (Lt - 1, Lz - 1, Ly - 1 - (k % Ly), 0)]
    out = []
    for t, z, y, x in raw:
        if parity is not None and (t + z + y + x) % 2 != parity:
            x = x - 1 if x > 0 else x + 1
        if (t, z, y, x) not in out:
            out.append((t, z, y, x))
    return out


def sites_for(L, n, seed, parity=None):
    forced = forced_sites(L, parity)
    rnd = [s for s in SM.sample_sites(L, n + len(forced), seed, parity) if s not in forced][:n]
    return forced + rnd


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    log("generating", LAT)
    U = synth.su3_field(LAT, 0.2, 1001)
    ctx = L.lq_init(0)
    f = L.lq_gauge_load(ctx, LAT, torch.from_numpy(U).cuda())
    yield ctx, f, U
    L.lq_field_free(f)
    L.lq_finalize(ctx)


def _gather(t, sites):
    """Host copy of the sampled sites of every column of a device field."""
    import torch
    idx = [torch.tensor([s[k] for s in sites], device=t.device) for k in range(4)]
    return t[:, idx[0], idx[1], idx[2], idx[3]].cpu().numpy()  # (n_col, n_site, ...)


def test_tm_schur_fp32_12col(env):
    import torch
    ctx, f, U = env
    psi = synth.gaussian_spinor(LAT, 12, 2002)
    ev = (np.indices(LAT[::-1]).sum(axis=0) % 2 == 0)[..., None, None]
    psi = psi * ev
    x = torch.from_numpy(psi).cuda()
    act = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    out = L.lq_apply(ctx, act, f, L.LQ_OP_SCHUR, 32, x)
    torch.cuda.synchronize()
    sites = sites_for(LAT, NS, 11, parity=0)
    got = _gather(out, sites)
    amat = {}
    want = np.array([[SM.schur_at(U, psi[c], M, CSW, MU, s, amat=amat) for s in sites] for c in range(12)])
    err, smax = rel(got, want), site_max_rel(got, want)
    log("schur fp32 12 col sampled rel", err, "per-site max", smax, "sites", len(sites))
    assert err < 1e-6 and smax < SITE_TOL[32]


def test_tm_solve_fp32_12col(env):
    import torch
    ctx, f, U = env
    b = synth.point_sources(LAT)
    bd = torch.from_numpy(b).cuda()
    act = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    x, st = L.lq_solve(ctx, act, f, L.params(tol=1e-10, sloppy_bits=32), bd)
    log("solve", st)
    assert st["status"] == 0 and st["true_rel_res"] <= 1e-10
    xh = x.cpu().numpy()
    F = W.field_strength(U)
    for c in (0, 7):  # one column of each chirality
        r = b[c] - W.tm_clover(U, xh[c], M, CSW, MU, F=F)
        res = np.linalg.norm(r) / np.linalg.norm(b[c])
        log("column", c, "oracle true residual", res)
        assert res <= 1e-10


def test_tm_multigrid_solve_12col(env):
    """The bench's multigrid propagator (4^4 aggregates, 24 vectors, FP32 V-cycles
    with the coarse stencil on the matrix cores): 1e-10 with the whole-lattice
    oracle operator on one column of each chirality."""
    import torch
    ctx, f, U = env
    b = synth.point_sources(LAT)
    bd = torch.from_numpy(b).cuda()
    act = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    st = L.lq_mg_setup(ctx, act, f, L.mg_params(block=(4, 4, 4, 4), n_vec=24, seed=11))
    log("multigrid setup", st)
    x, st = L.lq_solve(ctx, act, f, L.params(tol=1e-10, solver=3, maxiter=300), bd)
    log("multigrid solve", st)
    assert st["status"] == 0 and st["true_rel_res"] <= 1e-10
    xh = x.cpu().numpy()
    F = W.field_strength(U)
    for c in (1, 8):
        r = b[c] - W.tm_clover(U, xh[c], M, CSW, MU, F=F)
        res = np.linalg.norm(r) / np.linalg.norm(b[c])
        log("column", c, "oracle true residual", res)
        assert res <= 1e-10


def test_overlap_hw_fp16_12col(env):
    import torch
    ctx, f, U = env
    psi = synth.gaussian_spinor(LAT, 12, 2003)
    # H_W needs only rho; the polynomial fields must still be valid
    act = L.action(L.LQ_OVERLAP, m=0.015, rho=1.5, cheb_N=4, cheb_a=0.3, cheb_b=48.0)
    out = L.lq_apply(ctx, act, f, L.LQ_OP_HW, 16, torch.from_numpy(psi).cuda())
    torch.cuda.synchronize()
    sites = sites_for(LAT, NS, 12)
    got = _gather(out, sites)
    want = np.array([[SM.hw_at(U, psi[c], 1.5, s) for s in sites] for c in range(12)])
    err, smax = rel(got, want), site_max_rel(got, want)
    log("H_W fp16 12 col sampled rel", err, "per-site max", smax, "sites", len(sites))
    assert err < 3e-3 and smax < SITE_TOL[16]


HLAT = (32, 32, 32, 96)
HISQ_MASSES = [0.002 * 25.0 ** (i / 7.0) for i in range(8)]


@pytest.fixture(scope="module")
def hisq_env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    log("generating HISQ fields", HLAT)
    V, Wl = synth.hisq_fields(HLAT, 2001)
    ctx = L.lq_init(0)
    fh = L.lq_hisq_load(ctx, HLAT, torch.from_numpy(V).cuda(), torch.from_numpy(Wl).cuda())
    yield ctx, fh, V, Wl
    L.lq_field_free(fh)
    L.lq_finalize(ctx)


def test_hisq_normal_fp16_12col(hisq_env):
    import torch
    ctx, fh, V, Wl = hisq_env
    chi = synth.gaussian_colour(HLAT, 12, 2004)
    ev = (np.indices(HLAT[::-1]).sum(axis=0) % 2 == 0)[..., None]
    chi = chi * ev
    out = L.lq_apply(ctx, L.action(L.LQ_HISQ, m=0.002), fh, L.LQ_OP_NORMAL_EVEN, 16, torch.from_numpy(chi).cuda())
    torch.cuda.synchronize()
    sites = sites_for(HLAT, NS, 13, parity=0)
    got = _gather(out, sites)
    want = np.array([[SM.even_normal_at(V, Wl, chi[c], 0.002, s) for s in sites] for c in range(12)])
    err, smax = rel(got, want), site_max_rel(got, want)
    log("HISQ M_e fp16 12 col sampled rel", err, "per-site max", smax, "sites", len(sites))
    assert err < 3e-3 and smax < SITE_TOL[16]


def test_hisq_multishift_8mass_solve(hisq_env):
    """The benchmark's HISQ solve (8 masses 0.002..0.05, 12 colour point
    sources at t = 0, 24, 48, 72, FP32 multi-shift + FP16 refinement): the
    whole-lattice oracle M_e(m) residual of one column at the lightest and the
    heaviest mass is <= 1e-10."""
    import torch
    from oracle import staggered as S
    ctx, fh, V, Wl = hisq_env
    b = synth.staggered_point_sources(HLAT, [0, 24, 48, 72])
    act = L.action(L.LQ_HISQ, m=HISQ_MASSES[0])
    x, st = L.lq_solve(ctx, act, fh, L.params(tol=1e-10, sloppy_bits=16, masses=HISQ_MASSES),
                       torch.from_numpy(b).cuda())
    log("hisq 8-mass solve", st)
    assert st["status"] == 0 and st["true_rel_res"] <= 1e-10
    ev = S.even_mask(HLAT)
    for i in (0, len(HISQ_MASSES) - 1):
        m = HISQ_MASSES[i]
        y = x[i, 5].cpu().numpy()
        be = b[5] * ev
        r = be - S.even_normal(V, Wl, y * ev, m)
        res = float(np.linalg.norm(r) / np.linalg.norm(be))
        log("mass", m, "column 5 oracle residual", res)
        assert res <= 1e-10


def test_overlap_sign_properties_fp32(env):
    """The order-200 sign function at full size: eps(H)^2 = 1 and eps(H)
    Hermitian, to the polynomial error plus FP32 rounding (properties that
    hold at any size; the sign function has no per-site evaluation)."""
    import torch
    ctx, f, U = env
    lo, hi = L.lq_hw_bounds(ctx, L.action(L.LQ_OVERLAP, m=0.015, rho=1.5), f, 200)
    a, b = 0.9 * lo * lo, 1.1 * hi * hi
    act = L.action(L.LQ_OVERLAP, m=0.015, rho=1.5, cheb_N=200, cheb_a=a, cheb_b=b)
    v = torch.from_numpy(synth.gaussian_spinor(LAT, 2, 2005)).cuda()
    y = L.lq_apply(ctx, act, f, L.LQ_OP_SIGN, 32, v)
    z = L.lq_apply(ctx, act, f, L.LQ_OP_SIGN, 32, y)
    torch.cuda.synchronize()
    sq = float(torch.linalg.vector_norm(z - v) / torch.linalg.vector_norm(v))
    d01 = complex(torch.vdot(v[0].flatten(), y[1].flatten()))
    d10 = complex(torch.vdot(y[0].flatten(), v[1].flatten()))
    herm = abs(d01 - d10) / (float(torch.linalg.vector_norm(v[0])) * float(torch.linalg.vector_norm(v[1])))
    log("eps^2 - 1:", sq, "hermiticity:", herm, "interval", a, b)
    assert sq < 1e-4
    assert herm < 1e-5
