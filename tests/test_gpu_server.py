"""Continuous-batching server through the C ABI.

Each request's columns must solve the system to the FP64 target (checked with
the oracle operator) and agree with the same columns solved alone by
lq_solve, whatever other requests ran beside them: requests of different
sizes join a running batch and leave it at iteration boundaries, and
twisted-clover and HISQ engines run at the same time on their own streams.
"""
import numpy as np
import pytest

import synth
from oracle import staggered as S
from oracle import solve as OS
from oracle import wilson as W
from paper_2201_09004_amd import lq as L

pytestmark = pytest.mark.gpu

M, CSW, MU = -0.0695, 1.0509, 0.01


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = L.lq_init(0)
    yield c
    L.lq_finalize(c)


def _resid(apply, x, b):
    return max(OS.rel_residual(apply, xi, bi) for xi, bi in zip(x, b))


def test_server_mixed_requests(ctx):
    Lw = (4, 4, 6, 8)
    U = synth.su3_field(Lw, 0.2, 91)
    fw = L.lq_gauge_load(ctx, Lw, U)
    Ls = (4, 4, 4, 8)
    V, Wl = synth.hisq_fields(Ls, 101)
    fh = L.lq_hisq_load(ctx, Ls, V, Wl)
    srv = None
    try:
        tm = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
        prm = L.params(tol=1e-10, sloppy_bits=32)
        bw = synth.point_sources(Lw)
        # twisted-clover requests of 5, 4 and 3 columns into an 8-slot engine:
        # the 4-column request must wait for slots, the 3-column one joins at once
        sizes = [(0, 5), (5, 9), (9, 12)]
        bs = [np.ascontiguousarray(bw[a:b]) for a, b in sizes]
        xs = [np.zeros_like(b) for b in bs]
        sts = [L.lq_stats() for _ in bs]
        # HISQ requests at two masses (two engines)
        bh = synth.staggered_point_sources(Ls, [0], colours=(0, 1, 2))
        ms = [0.05, 0.1]
        hx = [np.zeros_like(bh) for _ in ms]
        hst = [L.lq_stats() for _ in ms]
        srv = L.lq_server_create(ctx, 0, 8)
        tickets = []
        for b, x, st in zip(bs, xs, sts):
            tickets.append(L.lq_submit(srv, tm, fw, prm, b, x, st))
        for mi, x, st in zip(ms, hx, hst):
            tickets.append(L.lq_submit(srv, L.action(L.LQ_HISQ, m=mi), fh, L.params(tol=1e-10, sloppy_bits=16),
                                       bh, x, st))
        for t in tickets:
            L.lq_wait(srv, t)
            assert L.lq_poll(srv, t)
        p50, p99, sps = L.lq_server_stats(srv)
        assert 0 < p50 <= p99 and sps > 0

        F = W.field_strength(U)
        Dtm = lambda v: W.tm_clover(U, v, M, CSW, MU, F=F)  # noqa: E731
        for b, x, st in zip(bs, xs, sts):
            d = st.as_dict()
            assert d["status"] == 0 and d["true_rel_res"] <= 1e-10, d
            assert _resid(Dtm, x, b) < 1e-10
            alone, sa = L.lq_solve(ctx, tm, fw, prm, b)
            assert sa["status"] == 0
            assert rel(x, alone) < 1e-8
        ev = S.even_mask(Ls)
        for mi, x, st in zip(ms, hx, hst):
            d = st.as_dict()
            assert d["status"] == 0, d
            assert np.all(x[:, ~ev[..., 0]] == 0)
            assert _resid(lambda v: S.even_normal(V, Wl, v, mi), x, bh * ev) < 1e-10
            alone, sa = L.lq_solve(ctx, L.action(L.LQ_HISQ, m=mi), fh, L.params(tol=1e-10, sloppy_bits=16), bh)
            assert rel(x, alone) < 1e-8

        # a second wave reuses the resident engines
        x2 = np.zeros_like(bs[0])
        t = L.lq_submit(srv, tm, fw, prm, bs[0], x2)
        L.lq_wait(srv, t)
        assert rel(x2, xs[0]) < 1e-8
    finally:
        if srv is not None:
            L.lq_server_destroy(srv)
        L.lq_field_free(fw)
        L.lq_field_free(fh)


def test_server_rejections(ctx):
    Lw = (4, 4, 4, 4)
    U = synth.su3_field(Lw, 0.2, 5)
    f = L.lq_gauge_load(ctx, Lw, U)
    b = synth.point_sources(Lw)[:2]
    x = np.zeros_like(b)
    srv = L.lq_server_create(ctx, 0, 4)
    tiny = L.lq_server_create(ctx, 1, 4)
    try:
        with pytest.raises(L.LqError):  # Wilson is solved by lq_solve, not served
            L.lq_submit(srv, L.action(L.LQ_WILSON, m=0.1), f, L.params(), b, x)
        with pytest.raises(L.LqError):  # more columns than engine slots
            L.lq_submit(srv, L.action(L.LQ_TM_CLOVER, m=0.1, mu=0.01, c_sw=1.0), f, L.params(),
                        synth.point_sources(Lw)[:5], np.zeros((5,) + b.shape[1:], complex))
        t = L.lq_submit(tiny, L.action(L.LQ_TM_CLOVER, m=0.1, mu=0.01, c_sw=1.0), f, L.params(), b, x)
        with pytest.raises(L.LqError):  # engine larger than the 1-byte budget
            L.lq_wait(tiny, t)
    finally:
        L.lq_server_destroy(tiny)
        L.lq_server_destroy(srv)
        L.lq_field_free(f)


def test_budget_for_one_engine_makes_the_second_request_wait(ctx):
    """With an HBM budget that holds one engine but not two, a request for a
    second engine (another gauge field) waits until the first engine is idle
    and evicted, then completes with the result it has alone."""
    Lw = (4, 4, 4, 8)
    Ua, Ub = synth.su3_field(Lw, 0.2, 95), synth.su3_field(Lw, 0.2, 96)
    fa, fb = L.lq_gauge_load(ctx, Lw, Ua), L.lq_gauge_load(ctx, Lw, Ub)
    tm = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    prm = L.params(tol=1e-10, sloppy_bits=32)
    b = np.ascontiguousarray(synth.point_sources(Lw)[:4])
    srv = None
    try:
        # the smallest power-of-two budget that runs one engine: < 2 engines
        budget = 1 << 16
        while True:
            probe = L.lq_server_create(ctx, budget, 4)
            x = np.zeros_like(b)
            t = L.lq_submit(probe, tm, fa, prm, b, x)
            try:
                L.lq_wait(probe, t)
                ok = True
            except L.LqError as e:
                assert e.code == L.LQ_ENOMEM
                ok = False
            L.lq_server_destroy(probe)
            if ok:
                break
            budget *= 2
            assert budget < (1 << 34)
        srv = L.lq_server_create(ctx, budget, 4)
        xa, xb = np.zeros_like(b), np.zeros_like(b)
        sa, sb = L.lq_stats(), L.lq_stats()
        ta = L.lq_submit(srv, tm, fa, prm, b, xa, sa)
        tb = L.lq_submit(srv, tm, fb, prm, b, xb, sb)
        L.lq_wait(srv, ta)
        L.lq_wait(srv, tb)
        da, db = sa.as_dict(), sb.as_dict()
        assert da["status"] == 0 and db["status"] == 0
        # b waited for a: its latency covers a's solve and its own
        assert db["seconds"] > da["seconds"]
        for U, f, x in ((Ua, fa, xa), (Ub, fb, xb)):
            F = W.field_strength(U)
            assert _resid(lambda v: W.tm_clover(U, v, M, CSW, MU, F=F), x, b) < 1e-10
            alone, st = L.lq_solve(ctx, tm, f, prm, b)
            assert rel(x, alone) < 1e-8
    finally:
        if srv is not None:
            L.lq_server_destroy(srv)
        L.lq_field_free(fa)
        L.lq_field_free(fb)
