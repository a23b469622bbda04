"""GPU parity at the benchmark sizes, in the launch shapes the benchmark uses.

At 24^3 x 64 (twisted clover, overlap kernel) and 32^3 x 96 (HISQ) the oracle
is evaluated at sampled sites only (oracle.sampled, pinned against the
whole-lattice oracle on small lattices), except for the solver, whose FP64
true residual is computed with the whole-lattice oracle operator.  Inputs are
the benchmark's: links exp(i 0.2 H) seed 1001 and the Table 1 parameters;
12 Gaussian columns for operator checks, 12 point sources for the solve.
Tolerances as for the small lattices: relative L2 over the sampled outputs
1e-6 (FP32 storage) and 3e-3 (FP16 storage with per-site norms), 1e-10
relative true residual for the solution.
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


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


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
    sites = SM.sample_sites(LAT, NS, 11, parity=0)
    got = _gather(out, sites)
    amat = {}
    want = np.array([[SM.schur_at(U, psi[c], M, CSW, MU, s, amat=amat) for s in sites] for c in range(12)])
    err = rel(got, want)
    log("schur fp32 12 col sampled rel", err)
    assert err < 1e-6


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


def test_overlap_hw_fp16_12col(env):
    import torch
    ctx, f, U = env
    psi = synth.gaussian_spinor(LAT, 12, 2003)
    # H_W needs only rho; the polynomial fields must still be valid
    act = L.action(L.LQ_OVERLAP, m=0.015, rho=1.5, cheb_N=4, cheb_a=0.3, cheb_b=48.0)
    out = L.lq_apply(ctx, act, f, L.LQ_OP_HW, 16, torch.from_numpy(psi).cuda())
    torch.cuda.synchronize()
    sites = SM.sample_sites(LAT, NS, 12)
    got = _gather(out, sites)
    want = np.array([[SM.hw_at(U, psi[c], 1.5, s) for s in sites] for c in range(12)])
    err = rel(got, want)
    log("H_W fp16 12 col sampled rel", err)
    assert err < 3e-3


def test_hisq_normal_fp16_12col():
    import torch
    Lh = (32, 32, 32, 96)
    log("generating HISQ fields", Lh)
    V, Wl = synth.hisq_fields(Lh, 2001)
    chi = synth.gaussian_colour(Lh, 12, 2004)
    ev = (np.indices(Lh[::-1]).sum(axis=0) % 2 == 0)[..., None]
    chi = chi * ev
    ctx = L.lq_init(0)
    fh = L.lq_hisq_load(ctx, Lh, torch.from_numpy(V).cuda(), torch.from_numpy(Wl).cuda())
    try:
        out = L.lq_apply(ctx, L.action(L.LQ_HISQ, m=0.002), fh, L.LQ_OP_NORMAL_EVEN, 16,
                         torch.from_numpy(chi).cuda())
        torch.cuda.synchronize()
        sites = SM.sample_sites(Lh, NS, 13, parity=0)
        got = _gather(out, sites)
        want = np.array([[SM.even_normal_at(V, Wl, chi[c], 0.002, s) for s in sites] for c in range(12)])
        err = rel(got, want)
        log("HISQ M_e fp16 12 col sampled rel", err)
        assert err < 3e-3
    finally:
        L.lq_field_free(fh)
        L.lq_finalize(ctx)


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
