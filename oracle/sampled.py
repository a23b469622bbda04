"""Operators evaluated at a few chosen sites only (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  For checks at full
lattice sizes, where a whole-lattice FP64 application would take minutes,
each requested output site is computed straight from the definitions used by
the whole-lattice modules (`wilson`, `staggered`, `overlap`): the hopping sum
over the site's neighbours, the clover leaves around the site, and, for the
even-odd and even-site normal operators, the same sums nested over the
neighbours' neighbours.  The cost is proportional to the number of sampled
sites.  A site is a tuple (t, z, y, x); fields are indexed [t, z, y, x, ...].

Conventions are those of the whole-lattice modules: chiral gamma basis,
standard-sign Wilson operator (sec. 2.1, eq. 2), Luescher clover term
(eq. 3), twist i mu gamma5 (eq. 1), MILC staggered phases with fat and long
links (sec. 2.2, eq. 4), antiperiodic time for fermion fields.  The tests pin
every function here against the whole-lattice oracle on small lattices.
"""
from __future__ import annotations

import numpy as np

from .lattice import GAMMA, GAMMA5

EYE4 = np.eye(4, dtype=np.complex128)
EYE3 = np.eye(3, dtype=np.complex128)


def _ext(shape):
    Lt, Lz, Ly, Lx = shape[:4]
    return (Lx, Ly, Lz, Lt)


def step(L, site, mu, k):
    """(neighbour site, fermion boundary sign) of site + k * mu_hat."""
    t, z, y, x = site
    c = [x, y, z, t]
    v = c[mu] + k
    sign = 1.0
    if mu == 3 and (v < 0 or v >= L[3]):
        sign = -1.0
    c[mu] = v % L[mu]
    return (c[3], c[2], c[1], c[0]), sign


def parity_of(site):
    return sum(site) % 2


# ------------------------------------------------------------------ Wilson-type
def hop_at(U, psi, site, antiperiodic=True):
    """sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)] at x = site."""
    L = _ext(U.shape)
    out = np.zeros((4, 3), dtype=np.complex128)
    for mu in range(4):
        n, sg = step(L, site, mu, +1)
        sg = sg if antiperiodic else 1.0
        out += sg * (EYE4 - GAMMA[mu]) @ (psi[n] @ U[site][mu].T)
        n, sg = step(L, site, mu, -1)
        sg = sg if antiperiodic else 1.0
        out += sg * (EYE4 + GAMMA[mu]) @ (psi[n] @ U[n][mu].conj())
    return out


def wilson_at(U, psi, m, site, antiperiodic=True):
    """D_W(m) psi at one site."""
    return (4.0 + m) * psi[site] - 0.5 * hop_at(U, psi, site, antiperiodic)


def _link(U, site, mu, k=1):
    """U_mu(site) for k = +1; U_mu(site - mu)^dag for k = -1 (the link from site towards -mu)."""
    L = _ext(U.shape)
    if k == 1:
        return U[site][mu]
    n, _ = step(L, site, mu, -1)
    return U[n][mu].conj().T


def _path(U, site, moves):
    """Product of links along a closed path of unit moves (mu, +-1) starting at site."""
    L = _ext(U.shape)
    P = EYE3.copy()
    cur = site
    for mu, k in moves:
        P = P @ _link(U, cur, mu, k)
        cur, _ = step(L, cur, mu, k)
    return P


def field_strength_at(U, site):
    """F_{mu nu} at one site: (Q - Q^dag)/8 made traceless, Q the four leaves."""
    F = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Q = (_path(U, site, [(mu, 1), (nu, 1), (mu, -1), (nu, -1)])
                 + _path(U, site, [(nu, 1), (mu, -1), (nu, -1), (mu, 1)])
                 + _path(U, site, [(mu, -1), (nu, -1), (mu, 1), (nu, 1)])
                 + _path(U, site, [(nu, -1), (mu, 1), (nu, 1), (mu, -1)]))
            f = (Q - Q.conj().T) / 8.0
            F[(mu, nu)] = f - np.trace(f) / 3.0 * EYE3
    return F


def site_matrix_at(U, m, csw, mu_tw, site):
    """A(x) = (4+m) + C(x) + i mu gamma5 as a 12x12 matrix (index spin*3 + colour)."""
    A = (4.0 + m) * np.eye(12, dtype=np.complex128) + 1j * mu_tw * np.kron(GAMMA5, EYE3)
    if csw != 0.0:
        for (mu, nu), f in field_strength_at(U, site).items():
            A += -0.5 * csw * np.kron(GAMMA[mu] @ GAMMA[nu], f)
    return A


def _site_matrix(U, m, csw, mu_tw, site, amat):
    if amat is None:
        return site_matrix_at(U, m, csw, mu_tw, site)
    if site not in amat:
        amat[site] = site_matrix_at(U, m, csw, mu_tw, site)
    return amat[site]


def tm_clover_at(U, psi, m, csw, mu_tw, site, antiperiodic=True, amat=None):
    """Twisted-mass clover D psi at one site (amat: optional dict caching site matrices)."""
    A = _site_matrix(U, m, csw, mu_tw, site, amat)
    return (A @ psi[site].reshape(12)).reshape(4, 3) - 0.5 * hop_at(U, psi, site, antiperiodic)


def schur_at(U, psi_e, m, csw, mu_tw, site, antiperiodic=True, amat=None):
    """M_hat psi_e = psi_e - A_ee^-1 D_eo A_oo^-1 D_oe psi_e at one even site.

    D_eo / D_oe are the hopping blocks -1/2 hop restricted to the parities;
    only the even entries of psi_e are read.  amat: optional dict caching the
    site matrices (they do not depend on psi).
    """
    assert parity_of(site) == 0
    L = _ext(U.shape)
    cache = {}

    def u_odd(n):  # A(n)^-1 (D_oe psi_e)(n) at an odd site n
        if n not in cache:
            h = -0.5 * hop_at(U, psi_e, n, antiperiodic)
            A = _site_matrix(U, m, csw, mu_tw, n, amat)
            cache[n] = np.linalg.solve(A, h.reshape(12)).reshape(4, 3)
        return cache[n]

    acc = np.zeros((4, 3), dtype=np.complex128)
    for mu in range(4):
        n, sg = step(L, site, mu, +1)
        sg = sg if antiperiodic else 1.0
        acc += sg * (EYE4 - GAMMA[mu]) @ (u_odd(n) @ U[site][mu].T)
        n, sg = step(L, site, mu, -1)
        sg = sg if antiperiodic else 1.0
        acc += sg * (EYE4 + GAMMA[mu]) @ (u_odd(n) @ U[n][mu].conj())
    d = -0.5 * acc
    A = _site_matrix(U, m, csw, mu_tw, site, amat)
    return psi_e[site] - np.linalg.solve(A, d.reshape(12)).reshape(4, 3)


def hw_at(U, psi, rho, site, antiperiodic=True):
    """H_W psi = gamma5 D_W(-rho) psi at one site (sec. 2.3)."""
    return GAMMA5 @ wilson_at(U, psi, -rho, site, antiperiodic)


# ------------------------------------------------------------------ HISQ
def eta_at(site):
    """MILC phases eta_mu at one site (x, y, z, t order of mu)."""
    t, z, y, x = site
    return [(-1.0) ** t, (-1.0) ** (t + x), (-1.0) ** (t + x + y), 1.0]


def stag_hop_at(V, W, chi, site, antiperiodic=True):
    """1/2 sum_mu eta_mu [V chi(x+mu) - V^dag(x-mu) chi(x-mu) + W chi(x+3mu) - W^dag(x-3mu) chi(x-3mu)]."""
    L = _ext(V.shape)
    eta = eta_at(site)
    out = np.zeros(3, dtype=np.complex128)
    for mu in range(4):
        s = np.zeros(3, dtype=np.complex128)
        for k, links in ((1, V), (3, W)):
            n, sg = step(L, site, mu, k)
            sg = sg if antiperiodic else 1.0
            s += sg * links[site][mu] @ chi[n]
            n, sg = step(L, site, mu, -k)
            sg = sg if antiperiodic else 1.0
            s -= sg * links[n][mu].conj().T @ chi[n]
        out += eta[mu] * s
    return 0.5 * out


def even_normal_at(V, W, chi_e, m, site, antiperiodic=True):
    """M_e(m) chi_e = m^2 chi_e - D_eo D_oe chi_e at one even site."""
    assert parity_of(site) == 0
    L = _ext(V.shape)
    eta = eta_at(site)
    cache = {}

    def t_odd(n):  # (D_oe chi_e)(n): the hop at odd site n reads even sites only
        if n not in cache:
            cache[n] = stag_hop_at(V, W, chi_e, n, antiperiodic)
        return cache[n]

    acc = np.zeros(3, dtype=np.complex128)
    for mu in range(4):
        s = np.zeros(3, dtype=np.complex128)
        for k, links in ((1, V), (3, W)):
            n, sg = step(L, site, mu, k)
            sg = sg if antiperiodic else 1.0
            s += sg * links[site][mu] @ t_odd(n)
            n, sg = step(L, site, mu, -k)
            sg = sg if antiperiodic else 1.0
            s -= sg * links[n][mu].conj().T @ t_odd(n)
        acc += eta[mu] * s
    return m * m * chi_e[site] - 0.5 * acc


def sample_sites(L, n, seed, parity=None):
    """n distinct sites (t, z, y, x) drawn with a seeded generator, optionally of one parity."""
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(seed)
    out = []
    seen = set()
    while len(out) < n:
        s = (int(rng.integers(Lt)), int(rng.integers(Lz)), int(rng.integers(Ly)), int(rng.integers(Lx)))
        if parity is not None and parity_of(s) != parity:
            continue
        if s in seen:
            continue
        seen.add(s)
        out.append(s)
    return out
