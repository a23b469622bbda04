"""Wilson, clover and twisted-mass operators (oracle, FP64).

Paper sec. 2.1: eq. (2) defines the Wilson operator, eq. (1) the twisted-mass
action through a complex mass omega, eq. (3) adds the clover (Sheikholeslami-
Wohlert) term.  Readings used here (the paper's LaTeX is ambiguous):

* Sign (std).  Eq. (2) literally reads 1/2 sum (1 + eta gamma) U delta - (4+m).
  That operator equals -gamma5 D_W gamma5 for the standard
      D_W(m) = (4+m) - 1/2 sum_mu [(1-gamma_mu) U_mu(x) delta_{x+mu,y}
                                 + (1+gamma_mu) U_mu^dag(x-mu) delta_{x-mu,y}],
  which is what this module implements (`wilson_eq2_literal` keeps the literal
  form for the identity test).
* Twisted mass.  Re(omega) is the Wilson mass m and Im(omega) a twist mu on
  i*gamma5: D_tm = D_W(m) + i mu gamma5 (single flavour, tau3 = +1).
* Clover (std, Luescher normalisation).  C(x) = c_sw (i/4) sum_{mu,nu}
  sigma_{mu nu} F_{mu nu}(x) = -(c_sw/2) sum_{mu<nu} gamma_mu gamma_nu F_{mu nu},
  F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/8 made traceless, Q the sum of the four
  plaquette leaves around x.
"""
from __future__ import annotations

import numpy as np

from .lattice import GAMMA, GAMMA5, shift, site_matvec, site_matvec_dag, spin_mul, parity, dims

EYE4 = np.eye(4, dtype=np.complex128)


def hop(U, psi, antiperiodic=True):
    """sum_mu [(1-gamma_mu) U_mu(x) psi(x+mu) + (1+gamma_mu) U_mu^dag(x-mu) psi(x-mu)]."""
    out = np.zeros_like(psi)
    for mu in range(4):
        Umu = U[..., mu, :, :]
        fwd = site_matvec(Umu, shift(psi, mu, +1, antiperiodic))
        bwd = site_matvec_dag(shift(Umu, mu, -1), shift(psi, mu, -1, antiperiodic))
        out += spin_mul(EYE4 - GAMMA[mu], fwd) + spin_mul(EYE4 + GAMMA[mu], bwd)
    return out


def wilson(U, psi, m, antiperiodic=True):
    """D_W(m) psi, standard sign (eq. 2 up to the gamma5 conjugation)."""
    return (4.0 + m) * psi - 0.5 * hop(U, psi, antiperiodic)


def wilson_eq2_literal(U, psi, m, antiperiodic=True):
    """Eq. (2) as printed: 1/2 sum_{mu,eta} (1+eta gamma_mu) U psi(x+eta mu) - (4+m) psi."""
    out = -(4.0 + m) * psi
    for mu in range(4):
        Umu = U[..., mu, :, :]
        fwd = site_matvec(Umu, shift(psi, mu, +1, antiperiodic))
        bwd = site_matvec_dag(shift(Umu, mu, -1), shift(psi, mu, -1, antiperiodic))
        out += 0.5 * (spin_mul(EYE4 + GAMMA[mu], fwd) + spin_mul(EYE4 - GAMMA[mu], bwd))
    return out


def gamma5(psi):
    return spin_mul(GAMMA5, psi)


def _mm(*ms):
    out = ms[0]
    for m in ms[1:]:
        out = np.einsum("...ab,...bc->...ac", out, m)
    return out


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def leaves(U, mu, nu):
    """Sum Q_{mu nu}(x) of the four counter-clockwise plaquettes in the (mu,nu) plane at x."""
    Um, Un = U[..., mu, :, :], U[..., nu, :, :]
    S = shift
    q = _mm(Um, S(Un, mu, 1), _dag(S(Um, nu, 1)), _dag(Un))
    Um_m = S(Um, mu, -1)                       # U_mu(x-mu)
    q = q + _mm(Un, _dag(S(S(Um, nu, 1), mu, -1)), _dag(S(Un, mu, -1)), Um_m)
    Un_n = S(Un, nu, -1)                       # U_nu(x-nu)
    q = q + _mm(_dag(Um_m), _dag(S(Un_n, mu, -1)), S(Um_m, nu, -1), Un_n)
    q = q + _mm(_dag(Un_n), S(Um, nu, -1), S(Un_n, mu, 1), _dag(Um))
    return q


def field_strength(U):
    """Dict (mu,nu) -> F_{mu nu}(x) for mu < nu: (Q - Q^dag)/8, made traceless."""
    F = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Q = leaves(U, mu, nu)
            f = (Q - _dag(Q)) / 8.0
            tr = np.trace(f, axis1=-2, axis2=-1) / 3.0
            F[(mu, nu)] = f - tr[..., None, None] * np.eye(3)
    return F


def clover(U, psi, csw, F=None):
    """C psi with C = -(c_sw/2) sum_{mu<nu} gamma_mu gamma_nu (x) F_{mu nu}."""
    if F is None:
        F = field_strength(U)
    out = np.zeros_like(psi)
    for (mu, nu), f in F.items():
        out += spin_mul(GAMMA[mu] @ GAMMA[nu], site_matvec(f, psi))
    return -0.5 * csw * out


def site_matrix(U, m, csw, mu_tw, F=None):
    """Site-local 12x12 term A(x) = (4+m) + C(x) + i mu gamma5, index spin*3+colour."""
    if F is None:
        F = field_strength(U)
    shp = U.shape[:4]
    A = np.zeros(shp + (4, 3, 4, 3), dtype=np.complex128)
    A += (4.0 + m) * np.einsum("st,ab->stab", EYE4, np.eye(3)).transpose(0, 2, 1, 3)
    A += 1j * mu_tw * np.einsum("st,ab->stab", GAMMA5, np.eye(3)).transpose(0, 2, 1, 3)
    for (mu, nu), f in F.items():
        A += -0.5 * csw * np.einsum("st,...ab->...satb", GAMMA[mu] @ GAMMA[nu], f)
    return A.reshape(shp + (12, 12))


def apply_site(A, psi):
    shp = psi.shape
    return np.einsum("...ij,...j->...i", A, psi.reshape(shp[:-2] + (12,))).reshape(shp)


def tm_clover(U, psi, m, csw, mu_tw, antiperiodic=True, F=None):
    """D psi = D_W(m) psi + C psi + i mu gamma5 psi (sec. 2.1, eq. 1 and 3)."""
    out = wilson(U, psi, m, antiperiodic)
    if csw != 0.0:
        out = out + clover(U, psi, csw, F)
    if mu_tw != 0.0:
        out = out + 1j * mu_tw * gamma5(psi)
    return out


def tm_clover_dag(U, psi, m, csw, mu_tw, antiperiodic=True, F=None):
    """D^dag = gamma5 D(-mu) gamma5 (gamma5-hermiticity of D_W + C)."""
    return gamma5(tm_clover(U, gamma5(psi), m, csw, -mu_tw, antiperiodic, F))


class EvenOdd:
    """Symmetric even-odd Schur complement of D = A + D_hop, D_hop = -1/2 hop.

    With A the site term and D_eo, D_oe the hopping blocks,
        M_hat = 1 - A_ee^{-1} D_eo A_oo^{-1} D_oe           (on even sites)
        b_hat = A_ee^{-1} (b_e - D_eo A_oo^{-1} b_o)
        x_o   = A_oo^{-1} (b_o - D_oe x_e).
    Site inverses come from numpy.linalg.inv of each 12x12 site matrix.
    """

    def __init__(self, U, m, csw, mu_tw, antiperiodic=True):
        self.U, self.ap = U, antiperiodic
        A = site_matrix(U, m, csw, mu_tw)
        self.Ainv = np.linalg.inv(A)
        p = parity(dims(U.shape))
        self.even = (p == 0)[..., None, None]
        self.odd = (p == 1)[..., None, None]

    def dhop(self, psi):
        return -0.5 * hop(self.U, psi, self.ap)

    def mhat(self, psi_e):
        psi_e = psi_e * self.even
        t = apply_site(self.Ainv, self.dhop(psi_e) * self.odd)
        u = apply_site(self.Ainv, self.dhop(t) * self.even)
        return (psi_e - u) * self.even

    def source(self, b):
        t = apply_site(self.Ainv, b * self.odd)
        return apply_site(self.Ainv, (b - self.dhop(t)) * self.even) * self.even

    def reconstruct(self, x_e, b):
        x_e = x_e * self.even
        x_o = apply_site(self.Ainv, (b - self.dhop(x_e)) * self.odd) * self.odd
        return x_e + x_o
