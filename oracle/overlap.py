"""Overlap operator through a Chebyshev approximation of the sign function (oracle).

Paper sec. 2.3: D_ov is built from D_w(-rho) / sqrt(D_w^dag D_w), rewritten as
gamma5 eps(H_W) with H_W = gamma5 D_w(-rho) and eps the matrix sign function;
eps is approximated by a Chebyshev polynomial (Fig. 2: deviation below 1e-5)
that is evaluated by Clenshaw's recursion on the GPU.  Readings:

* eps_N(H) v = H * P_N(H^2) v with P_N(y) = sum_{k=0}^{N} c_k T_k(Z(y)),
  Z(y) = (2y - (a+b)) / (b-a), approximating y^{-1/2} on [a, b] that holds the
  spectrum of H^2; the order N counts degrees in H^2 (2N+1 products with H).
  c_0 is stored already halved (no c_0/2 convention).
* Coefficients: Chebyshev interpolation of y^{-1/2} at the N+1 Chebyshev nodes
  of [a, b] (the paper's exchange iteration is a refinement of the same
  polynomial; the coefficients are an input to both sides).
* Normalisation: the printed 1/rho prefactor is read as rho (free-field
  continuum limit rho (1 + V) -> i gamma.p): D(0) = rho (1 + gamma5 eps(H_W)),
  massive D(m) = (rho - m/2)(1 + gamma5 eps(H_W)) + m.

The oracle evaluates the polynomial with the forward three-term recurrence
T_{k+1} = 2 Z T_k - T_{k-1}, a different route from the Clenshaw recursion
used by the GPU path.
"""
from __future__ import annotations

import numpy as np

from .lattice import GAMMA5, spin_mul
from .wilson import wilson


def hw(U, psi, rho, antiperiodic=True):
    """H_W psi = gamma5 D_W(-rho) psi (no clover)."""
    return spin_mul(GAMMA5, wilson(U, psi, -rho, antiperiodic))


def cheb_coeffs(a, b, N):
    """c_0..c_N of the degree-N Chebyshev interpolant of y^{-1/2} on [a, b]."""
    j = np.arange(N + 1)
    theta = np.pi * (j + 0.5) / (N + 1)
    y = 0.5 * (b - a) * np.cos(theta) + 0.5 * (b + a)
    f = 1.0 / np.sqrt(y)
    k = np.arange(N + 1)
    c = (2.0 / (N + 1)) * np.cos(np.outer(k, theta)) @ f
    c[0] *= 0.5
    return c


def cheb_eval_scalar(c, a, b, y):
    """P_N(y) = sum c_k T_k(Z(y)) for scalar/array y (numpy's chebval)."""
    z = (2.0 * np.asarray(y) - (a + b)) / (b - a)
    return np.polynomial.chebyshev.chebval(z, c)


def sign_deviation(c, a, b, n=20001):
    """max over x^2 in [a, b] of |x P_N(x^2) - sign(x)| = max |sqrt(y) P(y) - 1|."""
    y = np.linspace(a, b, n)
    return float(np.max(np.abs(np.sqrt(y) * cheb_eval_scalar(c, a, b, y) - 1.0)))


def sign_hw(U, psi, rho, c, a, b, antiperiodic=True):
    """eps_N(H_W) psi by the forward Chebyshev recurrence, then one product with H_W."""
    H = lambda v: hw(U, v, rho, antiperiodic)
    Z = lambda v: (2.0 * H(H(v)) - (a + b) * v) / (b - a)
    t_prev = psi
    acc = c[0] * psi
    if len(c) > 1:
        t_cur = Z(psi)
        acc = acc + c[1] * t_cur
        for k in range(2, len(c)):
            t_next = 2.0 * Z(t_cur) - t_prev
            acc = acc + c[k] * t_next
            t_prev, t_cur = t_cur, t_next
    return H(acc)


def overlap(U, psi, rho, m, c, a, b, antiperiodic=True):
    """D(m) psi = (rho - m/2)(psi + gamma5 eps(H_W) psi) + m psi."""
    e = spin_mul(GAMMA5, sign_hw(U, psi, rho, c, a, b, antiperiodic))
    return (rho - 0.5 * m) * (psi + e) + m * psi


def overlap_dag(U, psi, rho, m, c, a, b, antiperiodic=True):
    """D(m)^dag = gamma5 D(m) gamma5 (gamma5-hermiticity)."""
    return spin_mul(GAMMA5, overlap(U, spin_mul(GAMMA5, psi), rho, m, c, a, b, antiperiodic))


def hw_extremes(U, rho, antiperiodic=True, tol=1e-10):
    """(lambda_min, lambda_max) of |H_W| from ARPACK on H_W^2 (reference tool)."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    shp = U.shape[:4] + (4, 3)
    n = int(np.prod(shp))

    def mv(v):
        v = v.reshape(shp)
        return hw(U, hw(U, v, rho, antiperiodic), rho, antiperiodic).ravel()

    op = LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    lmax = eigsh(op, k=1, which="LA", tol=tol, return_eigenvectors=False)[0]
    lmin = eigsh(op, k=1, which="SA", tol=tol, return_eigenvectors=False)[0]
    return float(np.sqrt(lmin)), float(np.sqrt(lmax))


# ------------------------------------------------------------------ low modes (sec. 2.3)
def hw_low_modes_dense(U, rho, n, antiperiodic=True):
    """The n eigenpairs of H_W with the smallest |lambda| (dense numpy eigh;
    small lattices only).  Returns (lam[n], vecs[n][T,Z,Y,X,4,3]), |lam| ascending."""
    from .dense import wilson_tm_clover_dense
    from .lattice import GAMMA5 as G5
    D = wilson_tm_clover_dense(U, -rho, antiperiodic=antiperiodic)
    V = D.shape[0] // 12
    H = np.kron(np.eye(V), np.kron(G5, np.eye(3))) @ D
    w, Q = np.linalg.eigh(H)
    order = np.argsort(np.abs(w), kind="stable")[:n]
    shp = U.shape[:4] + (4, 3)
    return w[order], np.array([Q[:, i].reshape(shp) for i in order])


def sign_hw_projected(U, psi, rho, c, a, b, lam, vecs, antiperiodic=True):
    """eps(H_W) psi with the low modes (lam, vecs) treated exactly and the
    Chebyshev approximation on the rest (sec. 2.3):
        eps psi = sum_i sign(lam_i) u_i <u_i, psi> + P eps_N(H_W) P psi,
    P = 1 - sum_i u_i u_i^dag (the projection is applied on both sides of
    the polynomial, which maps the projected space to itself only exactly)."""
    def proj(v):
        out = v.copy()
        for u in vecs:
            out = out - u * np.vdot(u, v)
        return out
    low = sum(np.sign(l) * u * np.vdot(u, psi) for l, u in zip(lam, vecs))
    return low + proj(sign_hw(U, proj(psi), rho, c, a, b, antiperiodic))
