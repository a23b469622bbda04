"""Pins of the multigrid oracle (oracle/multigrid.py) by facts other than itself:
orthonormality of the aggregated basis, the free-field block average (a closed
form: the Galerkin operator of constant block vectors is a Wilson operator on
the coarse lattice with hopping 1/b and a shifted mass), exactness of the
two-level method when the aggregated basis spans the whole space, the
nearest-neighbour structure of the Galerkin operator and its gamma5-
hermiticity."""
import numpy as np
import pytest

import synth
from oracle import lattice as lat
from oracle import multigrid as MG
from oracle import wilson as W


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_basis_orthonormal_and_restrict_prolong_identity():
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    vecs = synth.gaussian_spinor(L, nv, 501)
    Q = MG.block_orthonormalize(vecs, block)
    for X in range(Q.shape[0]):
        for s in range(2):
            G = Q[X, s].conj() @ Q[X, s].T
            assert np.abs(G - np.eye(nv)).max() < 1e-13
    rng = np.random.default_rng(502)
    vc = rng.standard_normal(Q.shape[:3]) + 1j * rng.standard_normal(Q.shape[:3])
    assert _rel(MG.restrict(Q, MG.prolong(Q, vc, L, block), L, block), vc) < 1e-14
    # the first vector lies in the span on every aggregate: P R w_0 = w_0
    w0 = vecs[0]
    assert _rel(MG.prolong(Q, MG.restrict(Q, w0, L, block), L, block), w0) < 1e-13
    # chirality is kept apart: the prolongation of a chirality-(+) coarse vector has no (-) components
    vp = vc.copy()
    vp[:, 1, :] = 0.0
    f = MG.prolong(Q, vp, L, block)
    assert np.abs(f[..., 2:, :]).max() == 0.0


def test_free_field_block_average_is_a_coarse_wilson_operator():
    """U = 1 and the twelve constant spin-colour vectors: every aggregate of b^4
    sites is averaged exactly, and R D P = (4 + m - 4(b-1)/b) - 1/(2b) H_c + i mu
    gamma5 with H_c the free hopping term of the coarse lattice (the internal
    bonds of a block add to the mass term, the b^3 bonds through a face carry
    weight 1/b)."""
    L, b = (4, 4, 4, 8), 2
    block = (b, b, b, b)
    U = synth.unit_gauge(L)
    vecs = np.zeros((6,) + lat.coords(L)[0].shape + (4, 3), dtype=np.complex128)
    for j in range(6):
        vecs[j].reshape(-1, 12)[:, j] = 1.0
        vecs[j].reshape(-1, 12)[:, 6 + j] = 1.0
    Q = MG.block_orthonormalize(vecs, block)
    m, csw, mu = -0.3, 1.0, 0.2
    Lc = MG.coarse_dims(L, block)
    Vc = int(np.prod(Lc))
    rng = np.random.default_rng(503)
    vc = rng.standard_normal((Vc, 2, 6)) + 1j * rng.standard_normal((Vc, 2, 6))
    got = MG.coarse_apply(U, Q, block, vc, m, csw, mu)
    # coarse index (s, j) is spin-colour component 6 s + j
    Uc = synth.unit_gauge(Lc)
    fc = vc.reshape((Lc[3], Lc[2], Lc[1], Lc[0], 4, 3))
    want = (4.0 + m - 4.0 * (b - 1) / b) * fc - W.hop(Uc, fc) / (2.0 * b) + 1j * mu * W.gamma5(fc)
    assert _rel(got.reshape(want.shape), want) < 1e-13


def test_full_rank_basis_makes_the_two_level_solve_exact():
    """With one site per aggregate and six vectors per chirality the basis is
    unitary, so P D_c^{-1} R b solves D x = b."""
    L, block = (2, 2, 2, 4), (1, 1, 1, 1)
    U = synth.su3_field(L, 0.3, 504)
    vecs = synth.gaussian_spinor(L, 6, 505)
    Q = MG.block_orthonormalize(vecs, block)
    m, csw, mu = -0.2, 1.0, 0.1
    Dc = MG.coarse_dense(U, Q, block, m, csw, mu)
    bsrc = synth.gaussian_spinor(L, 1, 506)[0]
    xc = np.linalg.solve(Dc, MG.restrict(Q, bsrc, L, block).ravel())
    x = MG.prolong(Q, xc.reshape(Q.shape[:3]), L, block)
    assert _rel(W.tm_clover(U, x, m, csw, mu), bsrc) < 1e-12


def test_galerkin_operator_structure():
    """D_c couples an aggregate only to itself and its 8 neighbours, and
    D_c(mu)^dag = Gamma5 D_c(-mu) Gamma5 with Gamma5 = diag(+1, -1) over the
    chirality index."""
    L, block, nv = (6, 4, 4, 8), (2, 2, 2, 2), 2
    U = synth.su3_field(L, 0.3, 507)
    vecs = synth.gaussian_spinor(L, nv, 508)
    Q = MG.block_orthonormalize(vecs, block)
    m, csw, mu = -0.1, 1.2, 0.15
    Dc = MG.coarse_dense(U, Q, block, m, csw, mu)
    Lc = MG.coarse_dims(L, block)
    Vc = int(np.prod(Lc))
    k = 2 * nv
    C = np.array(np.unravel_index(np.arange(Vc), (Lc[3], Lc[2], Lc[1], Lc[0]))).T[:, ::-1]  # (x, y, z, t)
    for Y in range(Vc):
        for X in range(Vc):
            d = [min((C[Y][i] - C[X][i]) % Lc[i], (C[X][i] - C[Y][i]) % Lc[i]) for i in range(4)]
            blk = Dc[Y * k:(Y + 1) * k, X * k:(X + 1) * k]
            if sum(d) > 1:
                assert np.abs(blk).max() == 0.0
            else:
                assert np.abs(blk).max() > 1e-3
    Dm = MG.coarse_dense(U, Q, block, m, csw, -mu)
    g5 = np.tile(np.repeat([1.0, -1.0], nv), Vc)
    assert np.abs(Dc.conj().T - g5[:, None] * Dm * g5[None, :]).max() < 1e-13
