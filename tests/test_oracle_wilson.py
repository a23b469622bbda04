"""Pins for the Wilson / clover / twisted-mass oracle (CPU only).

Each test fixes the oracle against something other than itself: Clifford
algebra, the free-field momentum-space closed form, the constant-field clover
closed form, gamma5-hermiticity, gauge covariance and brute-force dense solves.
"""
import numpy as np
import pytest

import synth
from oracle import lattice as lat
from oracle import wilson as W
from oracle import dense, solve


def test_gamma_algebra():
    g = lat.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4))
    assert np.allclose(lat.GAMMA5, np.diag([1, 1, -1, -1]))


def test_su3_generator():
    U = synth.su3_field((2, 2, 2, 4), 0.3, 5).reshape(-1, 3, 3)
    eye = np.einsum("nab,ncb->nac", U, U.conj())
    assert np.abs(eye - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    W3 = synth.u3_field((2, 2, 2, 4), 0.2, 6).reshape(-1, 3, 3)
    assert np.abs(np.einsum("nab,ncb->nac", W3, W3.conj()) - np.eye(3)).max() < 1e-13
    assert np.abs(np.abs(np.linalg.det(W3)) - 1).max() < 1e-13
    assert np.abs(np.linalg.det(W3) - 1).max() > 1e-3   # a genuine U(1) part


def _plane_wave(L, p, u):
    x, y, z, t = lat.coords(L)
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * u


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 3, 1), (3, 1, 0, 6)])
def test_free_field_closed_form(n):
    """U = 1: D(p) = m + sum(1 - cos p) + i sum gamma sin p; p_t = (2n+1) pi / T."""
    L = (4, 4, 4, 8)
    m, mu_tw = 0.1, 0.07
    p = [2 * np.pi * n[i] / L[i] for i in range(3)] + [(2 * n[3] + 1) * np.pi / L[3]]
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = _plane_wave(L, p, u)
    U = synth.unit_gauge(L)
    Dp = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) \
        + 1j * sum(lat.GAMMA[k] * np.sin(p[k]) for k in range(4)) + 1j * mu_tw * lat.GAMMA5
    got = W.tm_clover(U, psi, m, 1.3, mu_tw)     # clover vanishes on the free field
    want = _plane_wave(L, p, Dp @ u)
    assert np.abs(got - want).max() < 1e-13
    # twisted mass: D^dag D = M^2 + s^2 + mu^2 on the free field
    M = m + sum(1 - np.cos(q) for q in p)
    s2 = sum(np.sin(q) ** 2 for q in p)
    dd = W.tm_clover_dag(U, W.tm_clover(U, psi, m, 0.0, mu_tw), m, 0.0, mu_tw)
    assert np.abs(dd - (M * M + s2 + mu_tw ** 2) * psi).max() < 1e-12


def test_eq2_literal_is_gamma5_conjugate():
    L = (4, 2, 2, 4)
    U = synth.su3_field(L, 0.3, 11)
    psi = synth.gaussian_spinor(L, 1, 12)[0]
    m = 0.2
    lit = W.wilson_eq2_literal(U, psi, m)
    std = -W.gamma5(W.wilson(U, W.gamma5(psi), m))
    assert np.abs(lit - std).max() < 1e-13


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_dense_loop_builder_agrees(L):
    U = synth.su3_field(L, 0.5, 21)
    psi = synth.gaussian_spinor(L, 1, 22)[0]
    m, csw, mu_tw = -0.3, 1.2, 0.15
    D = dense.wilson_tm_clover_dense(U, m, csw, mu_tw)
    got = (D @ psi.ravel()).reshape(psi.shape)
    want = W.tm_clover(U, psi, m, csw, mu_tw)
    assert np.abs(got - want).max() < 1e-12


def test_gamma5_hermiticity():
    L = (4, 4, 2, 4)
    U = synth.su3_field(L, 0.4, 31)
    phi, psi = synth.gaussian_spinor(L, 2, 32)
    m, csw = 0.05, 1.05
    D = lambda v, mu_tw: W.tm_clover(U, v, m, csw, mu_tw)
    # gamma5 (D_W + C) gamma5 = (D_W + C)^dag
    lhs = lat.dot(phi, W.gamma5(D(W.gamma5(psi), 0.0)))
    rhs = lat.dot(D(phi, 0.0), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    # twisted mass: gamma5 D(mu) gamma5 = D(-mu)^dag
    lhs = lat.dot(phi, W.gamma5(D(W.gamma5(psi), 0.3)))
    rhs = lat.dot(D(phi, -0.3), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_gauge_covariance():
    L = (4, 2, 4, 4)
    U = synth.su3_field(L, 0.4, 41)
    G = synth.random_gauge_transform(L, 42)
    psi = synth.gaussian_spinor(L, 1, 43)[0]
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = lat.shift(G, mu, 1)
        UG[..., mu, :, :] = np.einsum("...ab,...bc,...dc->...ad", G, U[..., mu, :, :], Gf.conj())
    Gpsi = np.einsum("...ab,...sb->...sa", G, psi)
    args = (0.1, 1.3, 0.2)
    lhs = W.tm_clover(UG, Gpsi, *args)
    rhs = np.einsum("...ab,...sb->...sa", G, W.tm_clover(U, psi, *args))
    assert np.abs(lhs - rhs).max() < 1e-12


def test_clover_constant_field_closed_form():
    """U_y(x) = exp(i theta x diag(1,-1,0)), other links 1: interior sites have
    eigenvalues (4+m) +- (c_sw/2) sin(theta) (x4 each) and (4+m) (x4)."""
    L = (6, 4, 4, 4)
    theta, m, csw = 0.37, 0.1, 1.7
    U = synth.unit_gauge(L)
    x, _, _, _ = lat.coords(L)
    d = np.exp(1j * theta * x[..., None] * np.array([1.0, -1.0, 0.0]))
    U[..., 1, :, :] = np.einsum("...a,ab->...ab", d, np.eye(3))
    A = W.site_matrix(U, m, csw, 0.0)
    for xi in range(1, L[0] - 1):
        ev = np.sort(np.linalg.eigvalsh(A[0, 0, 0, xi]))
        h = 0.5 * csw * np.sin(theta)
        want = np.sort([4 + m - h] * 4 + [4 + m] * 4 + [4 + m + h] * 4)
        assert np.abs(ev - want).max() < 1e-13


def test_clover_hermitian_chiral():
    L = (2, 2, 2, 4)
    U = synth.su3_field(L, 0.5, 51)
    A = W.site_matrix(U, 0.0, 1.3, 0.0).reshape(-1, 12, 12)
    assert np.abs(A - A.conj().transpose(0, 2, 1)).max() < 1e-14
    g5 = np.kron(lat.GAMMA5, np.eye(3))
    assert np.abs(A @ g5 - g5 @ A).max() < 1e-14


def test_brute_force_solve_2x4():
    L = (2, 2, 2, 2)
    U = synth.su3_field(L, 0.3, 61)
    b = synth.gaussian_spinor(L, 1, 62)[0]
    m, csw, mu_tw = 0.1, 1.0, 0.05
    D = dense.wilson_tm_clover_dense(U, m, csw, mu_tw)
    x_dense = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    x, _ = solve.bicgstab(lambda v: W.tm_clover(U, v, m, csw, mu_tw), b, tol=1e-13)
    assert np.abs(x - x_dense).max() < 1e-10 * np.abs(x_dense).max()
    x2, _ = solve.cgne(lambda v: W.tm_clover(U, v, m, csw, mu_tw),
                       lambda v: W.tm_clover_dag(U, v, m, csw, mu_tw), b, tol=1e-13)
    assert np.abs(x2 - x_dense).max() < 1e-10 * np.abs(x_dense).max()


def test_even_odd_schur_reconstructs_full_solution():
    L = (4, 4, 4, 4)
    U = synth.su3_field(L, 0.2, 71)
    b = synth.gaussian_spinor(L, 1, 72)[0]
    m, csw, mu_tw = -0.0695, 1.0509, 0.01
    D = dense.wilson_tm_clover_dense(U, m, csw, mu_tw)
    x_dense = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    eo = W.EvenOdd(U, m, csw, mu_tw)
    bh = eo.source(b)
    xe, _ = solve.bicgstab(eo.mhat, bh, tol=1e-13)
    x = eo.reconstruct(xe, b)
    assert np.abs(x - x_dense).max() < 1e-9 * np.abs(x_dense).max()
