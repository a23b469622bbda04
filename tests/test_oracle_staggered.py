"""Pins for the HISQ staggered oracle (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import lattice as lat
from oracle import staggered as S
from oracle import dense, solve


def _plane(L, p, c):
    x, y, z, t = lat.coords(L)
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None] * c


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 3, 2, 2), (2, 1, 5, 3)])
def test_free_field_normal_operator(n):
    """V = c1, W = c3 (times 1): D^dag D e^{ipx} c = (m^2 + sum (c1 sin p + c3 sin 3p)^2) e^{ipx} c."""
    L = (6, 4, 8, 8)
    c1, c3, m = 9.0 / 8.0, -1.0 / 24.0, 0.05
    p = [2 * np.pi * n[i] / L[i] for i in range(3)] + [(2 * n[3] + 1) * np.pi / L[3]]
    V = c1 * synth.unit_gauge(L)
    Wl = c3 * synth.unit_gauge(L)
    rng = np.random.default_rng(3)
    col = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    chi = _plane(L, p, col)
    got = S.hisq_dag(V, Wl, S.hisq(V, Wl, chi, m), m)
    lam = m * m + sum((c1 * np.sin(q) + c3 * np.sin(3 * q)) ** 2 for q in p)
    assert np.abs(got - lam * chi).max() < 1e-13


def test_milc_chroma_relation():
    """Sec. 2.2: psi^Chroma = (-1)^{(t%2)((x+y+z)%2)+(x+y+z+t)%2} psi^QUDA, Chroma mass sign flipped."""
    L = (4, 4, 4, 6)
    V, Wl = synth.hisq_fields(L, 81)
    chi = synth.gaussian_colour(L, 1, 82)[0]
    m = 0.0102
    s = S.chroma_sign(L)[..., None]
    lhs = s * S.hisq(V, Wl, s * chi, m)
    rhs = -S.chroma_op(V, Wl, chi, m)
    assert np.abs(lhs - rhs).max() < 1e-13
    # the MILC and CPS phases are genuinely different conventions
    assert np.abs(S.hop(V, Wl, chi) - S.hop(V, Wl, chi, convention="cps")).max() > 0.1


def test_epsilon_hermiticity():
    L = (4, 4, 4, 4)
    V, Wl = synth.hisq_fields(L, 91)
    phi, chi = synth.gaussian_colour(L, 2, 92)
    m = 0.03
    eps = ((-1.0) ** sum(lat.coords(L)))[..., None]
    assert np.abs(eps * S.hisq(V, Wl, eps * chi, m) - S.hisq_dag(V, Wl, chi, m)).max() < 1e-13
    lhs = lat.dot(phi, S.hisq_dag(V, Wl, chi, m))
    rhs = lat.dot(S.hisq(V, Wl, phi, m), chi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_gauge_covariance_fat_long():
    L = (4, 4, 4, 8)
    V, Wl = synth.hisq_fields(L, 101)
    G = synth.random_gauge_transform(L, 102)
    chi = synth.gaussian_colour(L, 1, 103)[0]
    VG, WG = np.empty_like(V), np.empty_like(Wl)
    for mu in range(4):
        VG[..., mu, :, :] = np.einsum("...ab,...bc,...dc->...ad", G, V[..., mu, :, :],
                                      lat.shift(G, mu, 1).conj())
        WG[..., mu, :, :] = np.einsum("...ab,...bc,...dc->...ad", G, Wl[..., mu, :, :],
                                      lat.shift(G, mu, 3).conj())
    lhs = S.hisq(VG, WG, np.einsum("...ab,...b->...a", G, chi), 0.02)
    rhs = np.einsum("...ab,...b->...a", G, S.hisq(V, Wl, chi, 0.02))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_even_normal_is_schur_of_DdagD():
    L = (4, 4, 4, 4)
    V, Wl = synth.hisq_fields(L, 111)
    chi = synth.gaussian_colour(L, 1, 112)[0]
    m = 0.07
    ev = S.even_mask(L)
    chi_e = chi * ev
    want = S.hisq_dag(V, Wl, S.hisq(V, Wl, chi_e, m), m) * ev
    assert np.abs(S.even_normal(V, Wl, chi_e, m) - want).max() < 1e-13


def test_dense_and_brute_force_solve():
    L = (4, 4, 4, 4)
    V, Wl = synth.hisq_fields(L, 121)
    b = synth.gaussian_colour(L, 1, 122)[0]
    m = 0.05
    D = dense.hisq_dense(V, Wl, m)
    assert np.abs((D @ b.ravel()).reshape(b.shape) - S.hisq(V, Wl, b, m)).max() < 1e-13
    x_dense = np.linalg.solve(D, b.ravel()).reshape(b.shape)
    x, _ = solve.cgne(lambda v: S.hisq(V, Wl, v, m), lambda v: S.hisq_dag(V, Wl, v, m), b, tol=1e-13)
    assert np.abs(x - x_dense).max() < 1e-10 * np.abs(x_dense).max()


def test_shifted_solves_equal_single_mass():
    L = (4, 4, 4, 4)
    V, Wl = synth.hisq_fields(L, 131)
    b = synth.gaussian_colour(L, 1, 132)[0] * S.even_mask(L)
    masses = [0.05, 0.08, 0.2]
    m0 = masses[0]
    A = lambda v: S.even_normal(V, Wl, v, m0)
    xs = solve.shifted_solves(A, b, [mi * mi - m0 * m0 for mi in masses], tol=1e-13)
    for mi, xi in zip(masses, xs):
        assert solve.rel_residual(lambda v: S.even_normal(V, Wl, v, mi), xi, b) < 1e-12
