"""Plain FP64 reference solvers and residuals (oracle).

The solvers of the paper (BiCGStab, CG, multi-shift CG, sec. 2.1-2.3 and
Tables 2-3) all aim at the plain result x = D^{-1} b or x_i = (A + sigma_i)^{-1} b;
here they are written in their textbook form (no preconditioning, no mixed
precision, one right-hand side at a time) so that a GPU solution can be checked
by its true residual ||b - D x|| / ||b|| computed with the oracle operator.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _nrm(a):
    return float(np.linalg.norm(a.ravel()))


def rel_residual(apply_D, x, b):
    """||b - D x||_2 / ||b||_2 in FP64."""
    return _nrm(b - apply_D(x)) / _nrm(b)


def cg(apply_A, b, tol=1e-12, maxiter=10000, x0=None):
    """Conjugate gradient for Hermitian positive-definite A; returns (x, iters)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = _dot(r, r).real
    stop = (tol * _nrm(b)) ** 2
    for it in range(maxiter):
        if rr <= stop:
            return x, it
        Ap = apply_A(p)
        alpha = rr / _dot(p, Ap).real
        x += alpha * p
        r -= alpha * Ap
        rr_new = _dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxiter


def cgne(apply_D, apply_Ddag, b, tol=1e-12, maxiter=10000):
    """Solve D x = b by CG on D^dag D x = D^dag b."""
    rhs = apply_Ddag(b)
    return cg(lambda v: apply_Ddag(apply_D(v)), rhs, tol * 0.1, maxiter)


def bicgstab(apply_D, b, tol=1e-12, maxiter=10000):
    """Unpreconditioned BiCGStab (van der Vorst); returns (x, iters)."""
    x = np.zeros_like(b)
    r = b.copy()
    rhat = b.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    stop = tol * _nrm(b)
    for it in range(maxiter):
        rho_new = _dot(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_D(p)
        alpha = rho_new / _dot(rhat, v)
        s = r - alpha * v
        t = apply_D(s)
        omega = _dot(t, s) / _dot(t, t)
        x += alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        if _nrm(r) <= stop:
            return x, it + 1
    return x, maxiter


def shifted_solves(apply_A, b, sigmas, tol=1e-12, maxiter=10000):
    """x_i = (A + sigma_i)^{-1} b, one plain CG per shift."""
    return [cg(lambda v, s=s: apply_A(v) + s * v, b, tol, maxiter)[0] for s in sigmas]
