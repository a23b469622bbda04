"""Lattice geometry, gamma matrices and shifts for the oracle (FP64).

Arrays over the lattice are shaped (Lt, Lz, Ly, Lx, ...); direction mu = 0..3
is x, y, z, t and lives on array axis 3 - mu.  Space is periodic; time is
antiperiodic for fermion fields when `antiperiodic` is set (std: the paper does
not state its boundary conditions).
"""
from __future__ import annotations

import numpy as np

AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def gammas():
    """Euclidean gamma matrices gamma_1..gamma_4 in a chiral basis, shape (4,4,4).

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1,2,3),
    gamma_4 = [[0, 1], [1, 0]], so gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
    = diag(1, 1, -1, -1).
    """
    s = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k][0:2, 2:4] = -1j * s[k]
        g[k][2:4, 0:2] = 1j * s[k]
    g[3][0:2, 2:4] = np.eye(2)
    g[3][2:4, 0:2] = np.eye(2)
    return g


GAMMA = gammas()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]


def dims(field_shape):
    """(Lx, Ly, Lz, Lt) from an array whose first four axes are (Lt,Lz,Ly,Lx)."""
    Lt, Lz, Ly, Lx = field_shape[:4]
    return (Lx, Ly, Lz, Lt)


def coords(L):
    """Integer coordinate arrays x, y, z, t each of shape (Lt,Lz,Ly,Lx)."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly),
                             np.arange(Lx), indexing="ij")
    return x, y, z, t


def parity(L):
    x, y, z, t = coords(L)
    return (x + y + z + t) % 2


def shift(f, mu, k, antiperiodic=False):
    """g(x) = f(x + k*mu_hat) for a field f whose first 4 axes are the lattice.

    With `antiperiodic` and mu = t, values that crossed the time boundary are
    negated (fermion fields).  Gauge links are periodic: call with False.
    """
    out = np.roll(f, -k, axis=AXIS[mu])
    if antiperiodic and mu == 3 and k != 0:
        Lt = f.shape[0]
        t = np.arange(Lt)
        crossed = (t + k < 0) | (t + k >= Lt)
        out[crossed] *= -1.0
    return out


def site_matvec(U, v):
    """Colour matrix times colour vector at every site: U[...,a,b] v[...,s,b]."""
    return np.einsum("...ab,...sb->...sa", U, v)


def site_matvec_dag(U, v):
    return np.einsum("...ba,...sb->...sa", U.conj(), v)


def spin_mul(G, v):
    """Spin matrix G (4x4) applied to a spinor field v[..., spin, colour]."""
    return np.einsum("st,...ta->...sa", G, v)


def dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def norm(a):
    return float(np.linalg.norm(a.ravel()))
