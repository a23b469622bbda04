"""Pins for the Chebyshev sign function and overlap oracle (CPU only)."""
import numpy as np

import synth
from oracle import lattice as lat
from oracle import overlap as OV
from oracle import dense

RHO = 1.5


def _dense_hw(U, rho=RHO):
    D = dense.wilson_tm_clover_dense(U, -rho)
    V = D.shape[0] // 12
    g5 = np.kron(np.eye(V), np.kron(lat.GAMMA5, np.eye(3)))
    return g5 @ D


def test_cheb_coeffs_match_numpy_interpolant():
    """Interpolation coefficients equal numpy's Chebyshev interpolant of y^{-1/2}."""
    a, b, N = 0.3, 40.0, 60
    c = OV.cheb_coeffs(a, b, N)
    f = lambda z: 1.0 / np.sqrt(0.5 * (b - a) * z + 0.5 * (b + a))
    ref = np.polynomial.chebyshev.chebinterpolate(f, N)
    assert np.abs(c - ref).max() < 1e-13


def test_sign_scalar_reduction_2x4():
    """On the dense H_W at 2^4: eps_N(H) v from eigh + chebval equals the recurrence."""
    L = (2, 2, 2, 2)
    U = synth.su3_field(L, 0.2, 201)
    H = _dense_hw(U)
    w, Q = np.linalg.eigh(H)
    a, b = 0.9 * w.__abs__().min() ** 2, 1.1 * w.__abs__().max() ** 2
    c = OV.cheb_coeffs(a, b, 60)
    v = synth.gaussian_spinor(L, 1, 202)[0]
    fw = w * OV.cheb_eval_scalar(c, a, b, w * w)
    want = (Q @ (fw * (Q.conj().T @ v.ravel()))).reshape(v.shape)
    got = OV.sign_hw(U, v, RHO, c, a, b)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # within the approximation bound of the exact sign
    delta = OV.sign_deviation(c, a, b)
    exact = (Q @ (np.sign(w) * (Q.conj().T @ v.ravel()))).reshape(v.shape)
    assert lat.norm(got - exact) <= 1.01 * delta * lat.norm(v)


def test_order_200_meets_fig2_bound():
    """Fig. 2: deviation from sign(x) below 1e-5; at order 200 on a spectrum
    [0.6, 6.3] (smooth synthetic links) it is far below that."""
    a, b = 0.9 * 0.6 ** 2, 1.1 * 6.3 ** 2
    c = OV.cheb_coeffs(a, b, 200)
    assert OV.sign_deviation(c, a, b) < 1e-5
    assert OV.sign_deviation(c, a, b) < 1e-10


def test_free_field_overlap():
    """U = 1: D(0) = rho (1 + V(p)), V = (M + i gamma.s)/sqrt(M^2 + s^2), M = -rho + sum(1-cos p)."""
    L = (4, 4, 4, 4)
    U = synth.unit_gauge(L)
    ps = []
    for nx in range(4):
        for nt in range(2):
            ps.append([2 * np.pi * nx / 4, 0.0, 2 * np.pi / 4, (2 * nt + 1) * np.pi / 4])
    # spectrum bounds of H_W^2 = M^2 + s^2 over all lattice momenta
    ks = [2 * np.pi * k / 4 for k in range(4)]
    kt = [(2 * k + 1) * np.pi / 4 for k in range(4)]
    lam = [(-RHO + sum(1 - np.cos(q) for q in (a1, a2, a3, a4))) ** 2
           + sum(np.sin(q) ** 2 for q in (a1, a2, a3, a4))
           for a1 in ks for a2 in ks for a3 in ks for a4 in kt]
    a, b = 0.95 * min(lam), 1.05 * max(lam)
    c = OV.cheb_coeffs(a, b, 80)
    delta = OV.sign_deviation(c, a, b)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    x, y, z, t = lat.coords(L)
    for p in ps:
        ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None, None]
        M = -RHO + sum(1 - np.cos(q) for q in p)
        s = [np.sin(q) for q in p]
        Vp = (M * np.eye(4) + 1j * sum(lat.GAMMA[k] * s[k] for k in range(4))) / np.sqrt(M * M + sum(q * q for q in s))
        want = ph * (RHO * (np.eye(4) + Vp) @ u)
        got = OV.overlap(U, ph * u, RHO, 0.0, c, a, b)
        assert np.abs(got - want).max() < 10 * delta * np.abs(u).max() + 1e-12


def test_ginsparg_wilson_and_gamma5_hermiticity():
    L = (4, 2, 2, 4)
    U = synth.su3_field(L, 0.2, 211)
    a, b = 0.9 * 0.5 ** 2, 1.1 * 6.5 ** 2
    lo, hi = OV.hw_extremes(U, RHO)
    assert a < lo ** 2 and hi ** 2 < b
    c = OV.cheb_coeffs(a, b, 160)
    delta = OV.sign_deviation(c, a, b)
    assert delta < 1e-8
    psi, phi = synth.gaussian_spinor(L, 2, 212)
    g5 = lambda v: lat.spin_mul(lat.GAMMA5, v)
    D = lambda v: OV.overlap(U, v, RHO, 0.0, c, a, b)
    lhs = g5(D(psi)) + D(g5(psi))
    rhs = D(g5(D(psi))) / RHO
    assert lat.norm(lhs - rhs) < 50 * delta * lat.norm(psi)
    # a 1/rho prefactor would break it by O(1)
    Dalt = lambda v: D(v) / RHO ** 2
    bad = g5(Dalt(psi)) + Dalt(g5(psi)) - Dalt(g5(Dalt(psi))) / RHO
    assert lat.norm(bad) > 0.1 * lat.norm(psi)
    m = 0.015
    Dm = lambda v: OV.overlap(U, v, RHO, m, c, a, b)
    l1 = lat.dot(phi, g5(Dm(g5(psi))))
    r1 = lat.dot(Dm(phi), psi)
    assert abs(l1 - r1) < 1e-10 * abs(r1)


def test_overlap_eigenvalues_on_circle_2x4():
    """Brute force at 2^4: eigenvalues of rho (1 + gamma5 eps(H_W)) lie on |lambda - rho| = rho."""
    L = (2, 2, 2, 2)
    U = synth.su3_field(L, 0.3, 221)
    H = _dense_hw(U)
    w, Q = np.linalg.eigh(H)
    a, b = 0.9 * np.abs(w).min() ** 2, 1.1 * np.abs(w).max() ** 2
    c = OV.cheb_coeffs(a, b, 100)
    delta = OV.sign_deviation(c, a, b)
    n = H.shape[0]
    # build the oracle overlap column by column through its vector interface
    cols = []
    eye = np.eye(n, dtype=np.complex128)
    for j in range(n):
        cols.append(OV.overlap(U, eye[:, j].reshape(L[::-1] + (4, 3)), RHO, 0.0, c, a, b).ravel())
    Dov = np.array(cols).T
    ev = np.linalg.eigvals(Dov)
    assert np.abs(np.abs(ev - RHO) - RHO).max() < 10 * delta + 1e-10


def test_hw_extremes_matches_dense_spectrum_2x4():
    """The oracle's ARPACK interval equals the extreme |eigenvalues| of the
    dense H_W at 2^4 (numpy eigvalsh), so it can serve as the checker of the
    library's Lanczos interval."""
    L = (2, 2, 2, 2)
    for seed in (231, 232):
        U = synth.su3_field(L, 0.3, seed)
        H = _dense_hw(U)
        w = np.linalg.eigvalsh(H @ H)
        lo, hi = OV.hw_extremes(U, RHO)
        assert abs(lo - np.sqrt(w[0])) < 1e-8 * np.sqrt(w[0])
        assert abs(hi - np.sqrt(w[-1])) < 1e-8 * np.sqrt(w[-1])


def test_chiral_normal_operator_identity_2x4():
    """The identity behind the chirally projected overlap solve (sec. 2.3):
    with the exact sign function, on a vector of chirality s,
    D(m)^dag D(m) v = (1 - m^2/(4 rho^2)) 2 rho^2 (v + s P_s eps v) + m^2 v,
    and D(m) is normal.  Checked on the dense operator at 2^4."""
    L = (2, 2, 2, 2)
    U = synth.su3_field(L, 0.3, 241)
    H = _dense_hw(U)
    w, Q = np.linalg.eigh(H)
    eps = (Q * np.sign(w)) @ Q.conj().T
    n = H.shape[0]
    g5 = np.kron(np.eye(n // 12), np.kron(lat.GAMMA5, np.eye(3)))
    for m in (0.015, 0.1):
        D = (RHO - m / 2) * (np.eye(n) + g5 @ eps) + m * np.eye(n)
        N = D.conj().T @ D
        assert np.abs(N - D @ D.conj().T).max() < 1e-12
        v = synth.gaussian_spinor(L, 1, 242)[0].ravel()
        f = 1.0 - m * m / (4 * RHO * RHO)
        for s in (1, -1):
            P = 0.5 * (np.eye(n) + s * g5)
            vs = P @ v
            want = f * 2 * RHO ** 2 * (vs + s * P @ (eps @ vs)) + m * m * vs
            assert np.abs(N @ vs - want).max() < 1e-12 * np.abs(want).max()
            # the sector form as the solver evaluates it: p0 v + p1 (s e + g5 e), e = eps v
            e = eps @ vs
            alt = (f * 2 * RHO ** 2 + m * m) * vs + f * RHO ** 2 * (s * e + g5 @ e)
            assert np.abs(alt - want).max() < 1e-12 * np.abs(want).max()
        # masses are shifts of one operator: D(m)^dag D(m) = f (D(0)^dag D(0) + m^2 / f)
        D0 = RHO * (np.eye(n) + g5 @ eps)
        assert np.abs(N - f * (D0.conj().T @ D0 + m * m / f * np.eye(n))).max() < 1e-12


def test_golden_hw_spectra_come_from_the_oracle():
    """tests/golden/hw_spectra.json (the Chebyshev intervals of the GPU overlap
    tests) holds what the oracle computes: the 4^4 entry is recomputed here."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hw_spectra.json")
    with open(here) as f:
        t = json.load(f)
    e = t["4x4x4x4_eps0.2_seed311_rho1.5"]
    U = synth.su3_field(tuple(e["L"]), e["eps"], e["seed"])
    lo, hi = OV.hw_extremes(U, e["rho"], tol=1e-8)
    assert abs(lo - e["lmin"]) < 1e-7 * lo and abs(hi - e["lmax"]) < 1e-7 * hi


def test_low_mode_projected_sign_2x4():
    """Low-mode projection (sec. 2.3): with the n smallest |lambda| modes of
    H_W treated exactly, a Chebyshev interval that starts above them
    (0.9 lambda_{n+1}^2) gives the exact sign function within the polynomial
    bound, while the same polynomial without the projection does not (its
    interval misses the projected modes)."""
    L = (2, 2, 2, 2)
    U = synth.su3_field(L, 0.3, 251)
    H = _dense_hw(U)
    w, Q = np.linalg.eigh(H)
    lam, vecs = OV.hw_low_modes_dense(U, RHO, 25)
    order = np.argsort(np.abs(w))
    assert np.allclose(np.abs(lam), np.abs(w[order[:25]]), atol=1e-12)
    n = 24  # project 24, the 25th sets the interval
    a, b = 0.9 * lam[n] ** 2, 1.1 * np.abs(w).max() ** 2
    c = OV.cheb_coeffs(a, b, 80)
    delta = OV.sign_deviation(c, a, b)
    v = synth.gaussian_spinor(L, 1, 252)[0]
    exact = (Q @ (np.sign(w) * (Q.conj().T @ v.ravel()))).reshape(v.shape)
    got = OV.sign_hw_projected(U, v, RHO, c, a, b, lam[:n], vecs[:n])
    assert lat.norm(got - exact) <= 1.01 * delta * lat.norm(v) + 1e-12
    bad = OV.sign_hw(U, v, RHO, c, a, b)
    assert lat.norm(bad - exact) > 100 * delta * lat.norm(v)
    # the projected modes are eigenvectors: H u = lam u
    for l, u in zip(lam[:n], vecs[:n]):
        assert lat.norm(OV.hw(U, u, RHO) - l * u) < 1e-12
