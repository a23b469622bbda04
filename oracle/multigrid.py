"""Two-level aggregation multigrid pieces for the twisted-clover operator (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

Paper sec. 2.1 and Table 2 time a multigrid inverter for the twisted-clover
action whose subspace setup is reusable across solves; the paper leaves the
method to QUDA's adaptive aggregation multigrid (Clark et al., Babich et al.,
cited in the paper).  Readings of that method used here (std):

* Aggregates.  The lattice is split into blocks of b = (bx, by, bz, bt) sites;
  block X of the coarse lattice Lc = L / b holds the fine sites with
  floor(x_mu / b_mu) = X_mu.  Coarse sites are ordered lexicographically with
  x fastest.
* Prolongator.  Each near-null vector w_j (j = 0..Nv-1) is cut into aggregates
  and into its two chiral halves P_s w_j, P_s = (1 + s gamma5)/2, s = +1 (spins
  0, 1 in the chiral basis, coarse index 0) and s = -1 (spins 2, 3, coarse
  index 1).  On each (aggregate, chirality) the Nv pieces are orthonormalised
  in the order j = 0, 1, ... (Gram-Schmidt; here numpy's QR with the diagonal
  of R made real and positive, the same basis).  A coarse vector has
  components v_c[X, s, j]; (P v_c)(y) = sum_{s,j} v_c[X(y), s, j] q_{X,s,j}(y).
  Keeping the chiral halves apart makes P commute with gamma5, so the coarse
  operator inherits gamma5-hermiticity with Gamma5 = diag(+1, -1) over s.
* Restriction R = P^dag, so R P = 1.
* Coarse operator (Galerkin): D_c = R D P.  D couples nearest neighbours, so
  D_c couples each aggregate to itself and its eight neighbours.

The coarse operator here is the definition written out: D applied to the
prolongation of every coarse unit vector, then restricted (a dense matrix,
small lattices only).
"""
from __future__ import annotations

import numpy as np

from .lattice import dims
from .wilson import tm_clover


def coarse_dims(L, block):
    Lc = tuple(L[m] // block[m] for m in range(4))
    for m in range(4):
        if Lc[m] * block[m] != L[m]:
            raise ValueError("block must divide the lattice")
    return Lc


def _chiral_split(v):
    """(..., 4, 3) -> (..., 2, 6): chirality + (spins 0, 1), chirality - (spins 2, 3)."""
    shp = v.shape[:-2]
    return v.reshape(shp + (2, 6))


def _blocked(f, L, block):
    """Fine field (Lt,Lz,Ly,Lx, ...) -> (Vc, B, ...) with aggregates in coarse
    lexicographic order and the B sites of an aggregate in a fixed order."""
    Lx, Ly, Lz, Lt = L
    bx, by, bz, bt = block
    rest = f.shape[4:]
    g = f.reshape((Lt // bt, bt, Lz // bz, bz, Ly // by, by, Lx // bx, bx) + rest)
    # -> (ct, cz, cy, cx, bt, bz, by, bx, ...)
    nrest = len(rest)
    g = g.transpose((0, 2, 4, 6, 1, 3, 5, 7) + tuple(range(8, 8 + nrest)))
    return g.reshape(((Lt // bt) * (Lz // bz) * (Ly // by) * (Lx // bx), bt * bz * by * bx) + rest)


def _unblocked(g, L, block):
    Lx, Ly, Lz, Lt = L
    bx, by, bz, bt = block
    rest = g.shape[2:]
    nrest = len(rest)
    h = g.reshape((Lt // bt, Lz // bz, Ly // by, Lx // bx, bt, bz, by, bx) + rest)
    h = h.transpose((0, 4, 1, 5, 2, 6, 3, 7) + tuple(range(8, 8 + nrest)))
    return h.reshape((Lt, Lz, Ly, Lx) + rest)


def block_orthonormalize(vecs, block):
    """Near-null vectors vecs[Nv] (fine fields) -> Q of shape (Vc, 2, Nv, B*6):
    the orthonormal basis of every (aggregate, chirality)."""
    nv = vecs.shape[0]
    L = dims(vecs.shape[1:])
    coarse_dims(L, block)
    blk = np.stack([_chiral_split(_blocked(v, L, block)) for v in vecs])  # (Nv, Vc, B, 2, 6)
    Vc, B = blk.shape[1], blk.shape[2]
    Q = np.zeros((Vc, 2, nv, B * 6), dtype=np.complex128)
    for X in range(Vc):
        for s in range(2):
            A = blk[:, X, :, s, :].reshape(nv, B * 6).T  # columns = vectors
            q, r = np.linalg.qr(A)
            ph = np.diag(r) / np.abs(np.diag(r))
            Q[X, s] = (q * ph[None, :]).T
    return Q


def prolong(Q, vc, L, block):
    """Fine field from a coarse vector vc[Vc, 2, Nv]."""
    Vc, _, nv, n = Q.shape
    B = n // 6
    g = np.einsum("xsjk,xsj->xsk", Q, vc).reshape(Vc, 2, B, 6).transpose(0, 2, 1, 3)
    return _unblocked(g.reshape(Vc, B, 4, 3), L, block)


def restrict(Q, v, L, block):
    """Coarse vector R v = P^dag v, shape (Vc, 2, Nv)."""
    Vc, _, nv, n = Q.shape
    g = _chiral_split(_blocked(v, L, block))  # (Vc, B, 2, 6)
    g = g.transpose(0, 2, 1, 3).reshape(Vc, 2, n)
    return np.einsum("xsjk,xsk->xsj", Q.conj(), g)


def coarse_dense(U, Q, block, m, csw, mu_tw, antiperiodic=True):
    """D_c = R D P as a dense (Vc*2*Nv)^2 matrix (coarse index (X, s, j))."""
    L = dims(U.shape)
    Vc, _, nv, _ = Q.shape
    n = Vc * 2 * nv
    Dc = np.zeros((n, n), dtype=np.complex128)
    for k in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[k] = 1.0
        f = prolong(Q, e.reshape(Vc, 2, nv), L, block)
        Dc[:, k] = restrict(Q, tm_clover(U, f, m, csw, mu_tw, antiperiodic), L, block).ravel()
    return Dc


def coarse_apply(U, Q, block, vc, m, csw, mu_tw, antiperiodic=True):
    """D_c vc = R D P vc without forming D_c."""
    L = dims(U.shape)
    return restrict(Q, tm_clover(U, prolong(Q, vc, L, block), m, csw, mu_tw, antiperiodic), L, block)
