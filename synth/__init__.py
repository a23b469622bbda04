"""Seeded synthetic inputs for lattice Dirac-operator workloads.

This module is the only code shared by the CPU oracle and the GPU path.  It
holds no Dirac-operator arithmetic: it only draws random numbers and turns them
into gauge links and sources in the canonical host layout.

Canonical host layout (C order, FP64 complex):
  * site index s = x + Lx*(y + Ly*(z + Lz*t)); numpy arrays are shaped
    (Lt, Lz, Ly, Lx, ...) so that a flat view follows s;
  * gauge links  [V][4][3][3]: U_mu(x)[row][col], mu = 0..3 <-> x, y, z, t,
    the link from x to x + mu;
  * Wilson-type spinors [n_rhs][V][4][3] (spin, colour);
  * staggered colour vectors [n_rhs][V][3].

Random unitary links follow the workloads of the paper's ensembles (Table 1
shapes) with synthetic content: U = exp(i*eps*H), H = sum_a h_a lambda_a / 2
with h_a ~ N(0, 1) i.i.d. over the eight Gell-Mann matrices (SU(3)); for U(3)
an extra h_0 * 1/sqrt(6) is added to H.  The exponential is taken through the
eigendecomposition of H in FP64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann", "random_hermitian", "expi", "su3_field", "u3_field",
    "unit_gauge", "random_gauge_transform", "gaussian_spinor",
    "gaussian_colour", "point_sources", "staggered_point_sources",
    "hisq_fields", "lattice_shape", "volume",
]


def lattice_shape(L):
    """(Lt, Lz, Ly, Lx) for extents L = (Lx, Ly, Lz, Lt)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return (Lt, Lz, Ly, Lx)


def volume(L):
    return int(np.prod([int(v) for v in L]))


def gell_mann():
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
    return lam


def random_hermitian(rng, n, with_trace=False):
    """n Hermitian 3x3 matrices H = sum_a h_a lambda_a/2 (+ h_0/sqrt(6) * 1)."""
    h = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, gell_mann() / 2.0)
    if with_trace:
        h0 = rng.standard_normal(n)
        H = H + (h0 / np.sqrt(6.0))[:, None, None] * np.eye(3)
    return H


def expi(H, eps, chunk=1 << 20):
    """exp(i*eps*H) for a stack of Hermitian 3x3 matrices, via eigh, in chunks."""
    out = np.empty_like(H)
    for s in range(0, H.shape[0], chunk):
        w, Q = np.linalg.eigh(H[s:s + chunk])
        out[s:s + chunk] = np.einsum("nab,nb,ncb->nac", Q, np.exp(1j * eps * w), Q.conj())
    return out


def _link_field(L, eps, seed, with_trace):
    rng = np.random.default_rng(seed)
    n = volume(L) * 4
    U = expi(random_hermitian(rng, n, with_trace), eps)
    return U.reshape(lattice_shape(L) + (4, 3, 3))


def su3_field(L, eps, seed):
    """Gauge field of SU(3) links exp(i*eps*H), shape (Lt,Lz,Ly,Lx,4,3,3)."""
    return _link_field(L, eps, seed, with_trace=False)


def u3_field(L, eps, seed):
    """Field of U(3) links exp(i*eps*(H + h0/sqrt6)), same shape as su3_field."""
    return _link_field(L, eps, seed, with_trace=True)


def unit_gauge(L):
    U = np.zeros(lattice_shape(L) + (4, 3, 3), dtype=np.complex128)
    U[..., :, :, :] = np.eye(3)
    return U


def random_gauge_transform(L, seed, eps=1.5):
    """One SU(3) matrix per site, shape (Lt,Lz,Ly,Lx,3,3)."""
    rng = np.random.default_rng(seed)
    G = expi(random_hermitian(rng, volume(L)), eps)
    return G.reshape(lattice_shape(L) + (3, 3))


def gaussian_spinor(L, n_rhs, seed):
    """n_rhs Gaussian spinors: each of the 24 real components per site ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    shp = (n_rhs,) + lattice_shape(L) + (4, 3)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def gaussian_colour(L, n_rhs, seed):
    """n_rhs Gaussian staggered colour vectors, shape (n_rhs,Lt,Lz,Ly,Lx,3)."""
    rng = np.random.default_rng(seed)
    shp = (n_rhs,) + lattice_shape(L) + (3,)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def point_sources(L, origin=(0, 0, 0, 0)):
    """The 12 spin-colour point sources at one site: column k = 3*spin + colour."""
    x, y, z, t = origin
    b = np.zeros((12,) + lattice_shape(L) + (4, 3), dtype=np.complex128)
    for k in range(12):
        b[k, t, z, y, x, k // 3, k % 3] = 1.0
    return b


def staggered_point_sources(L, times, colours=(0, 1, 2), origin_xyz=(0, 0, 0)):
    """Colour point sources at the spatial origin for each time in `times`."""
    x, y, z = origin_xyz
    cols = [(t, c) for t in times for c in colours]
    b = np.zeros((len(cols),) + lattice_shape(L) + (3,), dtype=np.complex128)
    for k, (t, c) in enumerate(cols):
        b[k, t, z, y, x, c] = 1.0
    return b


def hisq_fields(L, seed, eps_fat=0.1, eps_long=0.2, naik=-1.0 / 24.0):
    """Coefficient-absorbed HISQ-like link fields (fat V, long W).

    V = exp(i*eps_fat*H) in SU(3) (near-unit); W = naik * exp(i*eps_long*H')
    in U(3) times the tree-level Naik coefficient.  Seeds seed and seed+1.
    """
    V = su3_field(L, eps_fat, seed)
    W = naik * u3_field(L, eps_long, seed + 1)
    return V, W
