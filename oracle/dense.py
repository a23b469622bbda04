"""Naive per-site loop builders of dense operator matrices (oracle, tiny lattices).

A second, deliberately plain route to the same operators as `wilson` and
`staggered`: Python loops over sites and directions, explicit coordinate
arithmetic for neighbours and boundary signs, explicit plaquette products for
the clover term.  Used for brute-force checks (dense solves, eigenvalues) at
2^4 and 4^4.  Row/column index = site * ncomp + component with site
s = x + Lx*(y + Ly*(z + Lz*t)) and component spin*3 + colour (Wilson) or
colour (staggered).
"""
from __future__ import annotations

import itertools

import numpy as np

from .lattice import GAMMA, GAMMA5


def _sites(L):
    Lx, Ly, Lz, Lt = L
    for t, z, y, x in itertools.product(range(Lt), range(Lz), range(Ly), range(Lx)):
        yield (x, y, z, t)


def _index(c, L):
    x, y, z, t = c
    Lx, Ly, Lz, _ = L
    return x + Lx * (y + Ly * (z + Lz * t))


def _step(c, mu, k, L):
    """Coordinates of c + k*mu (periodic) and the antiperiodic-time sign."""
    c = list(c)
    raw = c[mu] + k
    c[mu] = raw % L[mu]
    sign = -1.0 if (mu == 3 and (raw < 0 or raw >= L[3])) else 1.0
    return tuple(c), sign


def _link(U, c, mu):
    x, y, z, t = c
    return U[t, z, y, x, mu]


def _plaquette_sum(U, c, mu, nu, L):
    """Q_{mu nu}(c): four counter-clockwise leaves, built step by step."""
    dag = lambda m: m.conj().T
    total = np.zeros((3, 3), dtype=np.complex128)
    # each leaf: a sequence of (direction, forward?) moves around a plaquette
    paths = [[(mu, 1), (nu, 1), (mu, -1), (nu, -1)],
             [(nu, 1), (mu, -1), (nu, -1), (mu, 1)],
             [(mu, -1), (nu, -1), (mu, 1), (nu, 1)],
             [(nu, -1), (mu, 1), (nu, 1), (mu, -1)]]
    for path in paths:
        pos = c
        prod = np.eye(3, dtype=np.complex128)
        for d, f in path:
            if f > 0:
                prod = prod @ _link(U, pos, d)
                pos, _ = _step(pos, d, 1, L)
            else:
                pos, _ = _step(pos, d, -1, L)
                prod = prod @ dag(_link(U, pos, d))
        total += prod
    return total


def wilson_tm_clover_dense(U, m, csw=0.0, mu_tw=0.0, antiperiodic=True):
    """Dense D = D_W(m) + C + i mu gamma5 as a (12V, 12V) complex matrix."""
    Lt, Lz, Ly, Lx = U.shape[:4]
    L = (Lx, Ly, Lz, Lt)
    V = Lx * Ly * Lz * Lt
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    one4 = np.eye(4)
    for c in _sites(L):
        s = _index(c, L)
        blk = (4.0 + m) * np.eye(12) + 1j * mu_tw * np.kron(GAMMA5, np.eye(3))
        if csw != 0.0:
            for mu in range(4):
                for nu in range(mu + 1, 4):
                    Q = _plaquette_sum(U, c, mu, nu, L)
                    F = (Q - Q.conj().T) / 8.0
                    F = F - np.trace(F) / 3.0 * np.eye(3)
                    blk += -0.5 * csw * np.kron(GAMMA[mu] @ GAMMA[nu], F)
        D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += blk
        for mu in range(4):
            cf, sf = _step(c, mu, 1, L)
            sgn = sf if antiperiodic else 1.0
            n = _index(cf, L)
            D[12 * s:12 * s + 12, 12 * n:12 * n + 12] += \
                -0.5 * sgn * np.kron(one4 - GAMMA[mu], _link(U, c, mu))
            cb, sb = _step(c, mu, -1, L)
            sgn = sb if antiperiodic else 1.0
            n = _index(cb, L)
            D[12 * s:12 * s + 12, 12 * n:12 * n + 12] += \
                -0.5 * sgn * np.kron(one4 + GAMMA[mu], _link(U, cb, mu).conj().T)
    return D


def hisq_dense(V, W, m, antiperiodic=True):
    """Dense staggered D_MILC(m) with fat (1-hop) and long (3-hop) links, (3V, 3V)."""
    Lt, Lz, Ly, Lx = V.shape[:4]
    L = (Lx, Ly, Lz, Lt)
    N = Lx * Ly * Lz * Lt
    D = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    for c in _sites(L):
        x, y, z, t = c
        eta = [(-1) ** t, (-1) ** (t + x), (-1) ** (t + x + y), 1]
        s = _index(c, L)
        D[3 * s:3 * s + 3, 3 * s:3 * s + 3] += m * np.eye(3)
        for mu in range(4):
            for k, F in ((1, V), (3, W)):
                cf, sf = _step(c, mu, k, L)
                sgn = sf if antiperiodic else 1.0
                n = _index(cf, L)
                D[3 * s:3 * s + 3, 3 * n:3 * n + 3] += 0.5 * eta[mu] * sgn * _link(F, c, mu)
                cb, sb = _step(c, mu, -k, L)
                sgn = sb if antiperiodic else 1.0
                n = _index(cb, L)
                D[3 * s:3 * s + 3, 3 * n:3 * n + 3] -= \
                    0.5 * eta[mu] * sgn * _link(F, cb, mu).conj().T
    return D
