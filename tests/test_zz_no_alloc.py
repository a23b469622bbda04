"""The allocation-free entry point lq_apply_noalloc (packed vectors in the
library's fixed device scratch) against lq_apply_dev, the entry point that
allocates, through the C ABI: the same kernels, so the same bits.  Two calls
in a row, the second with a smaller input, so stale scratch contents from the
first cannot leak into the second; size and residency errors are refused."""
import numpy as np
import pytest

import synth
from paper_2201_09004_amd import lq as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = L.lq_init(0)
    yield c
    L.lq_finalize(c)


def _both(ctx, act, f, op, prec, x):
    import torch
    want = L.lq_apply(ctx, act, f, op, prec, x)  # tensors: lq_apply_dev (synchronises)
    got = torch.full_like(x, float("nan"))
    L.lq_apply_noalloc(ctx, act, f, op, prec, x, got)
    torch.cuda.synchronize()
    return want, got


@pytest.mark.parametrize("prec", [64, 32, 16])
def test_noalloc_wilson_type_matches_apply_dev(ctx, prec):
    import torch
    Lx = (6, 6, 4, 10)  # Vh = 720: a ragged last 64-site tile
    dev = torch.device("cuda:0")
    U = synth.su3_field(Lx, 0.2, 901)
    f = L.lq_gauge_load(ctx, Lx, U)
    psi = torch.from_numpy(synth.gaussian_spinor(Lx, 12, 902)).to(dev)
    try:
        cases = [(L.action(L.LQ_WILSON, m=0.1), L.LQ_OP_D), (L.action(L.LQ_WILSON, m=0.1), L.LQ_OP_DDAG),
                 (L.action(L.LQ_OVERLAP, m=0.015, rho=1.5, cheb_N=8), L.LQ_OP_HW)]
        if prec != 16:
            cases.append((L.action(L.LQ_TM_CLOVER, m=-0.0695, mu=0.01, c_sw=1.0509), L.LQ_OP_D))
        for act, op in cases:
            # 12 columns, then 5 (a smaller input into the same scratch)
            for n in (12, 5):
                x = psi[:n].contiguous()
                want, got = _both(ctx, act, f, op, prec, x)
                assert torch.equal(got, want), (act.kind, op, n)
    finally:
        L.lq_field_free(f)


def test_noalloc_hisq_matches_apply_dev(ctx):
    import torch
    Lx = (4, 4, 6, 8)
    dev = torch.device("cuda:0")
    V, Wl = synth.hisq_fields(Lx, 911)
    f = L.lq_hisq_load(ctx, Lx, V, Wl)
    chi = torch.from_numpy(synth.gaussian_colour(Lx, 12, 912)).to(dev)
    act = L.action(L.LQ_HISQ, m=0.0102)
    try:
        for prec in (32, 16):
            for op in (L.LQ_OP_D, L.LQ_OP_HOP):
                for n in (12, 3):
                    x = chi[:n].contiguous()
                    want, got = _both(ctx, act, f, op, prec, x)
                    assert torch.equal(got, want), (prec, op, n)
    finally:
        L.lq_field_free(f)


def test_noalloc_refuses_oversize_and_non_resident(ctx):
    import torch
    Lx = (8, 8, 8, 8)
    dev = torch.device("cuda:0")
    f = L.lq_gauge_load(ctx, Lx, synth.su3_field(Lx, 0.2, 921))
    act = L.action(L.LQ_WILSON, m=0.1)
    try:
        x = torch.from_numpy(synth.gaussian_spinor(Lx, 2, 922)).to(dev)
        out = torch.empty_like(x)
        # FP32 links of this field were never packed: refused, nothing allocated
        with pytest.raises(L.LqError) as e:
            L.lq_apply_noalloc(ctx, act, f, L.LQ_OP_D, 32, x, out)
        assert e.value.code == L.LQ_EINVAL and "not resident" in str(e.value)
        L.lq_apply(ctx, act, f, L.LQ_OP_D, 64, x)
        # 48 FP64 columns of 8^4 need 2 x 48 x 4096 x 192 B > 64 MiB
        big = torch.zeros((48,) + tuple(x.shape[1:]), dtype=x.dtype, device=dev)
        with pytest.raises(L.LqError) as e:
            L.lq_apply_noalloc(ctx, act, f, L.LQ_OP_D, 64, big, torch.empty_like(big))
        assert e.value.code == L.LQ_EINVAL and "scratch" in str(e.value)
        # an op outside the supported set
        with pytest.raises(L.LqError) as e:
            L.lq_apply_noalloc(ctx, act, f, L.LQ_OP_SIGN, 64, x, out)
        assert e.value.code == L.LQ_EINVAL
        # and the entry point still works after the refusals
        want, got = _both(ctx, act, f, L.LQ_OP_D, 64, x)
        assert torch.equal(got, want)
    finally:
        L.lq_field_free(f)
