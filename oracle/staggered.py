"""HISQ staggered operator (oracle, FP64).

Paper sec. 2.2, eq. (4): the staggered action after spin diagonalisation
psi = gamma_4^{x4} gamma_1^{x1} gamma_2^{x2} gamma_3^{x3} chi (MILC order)
leaves one colour vector per site with phases eta_mu(x); HISQ uses a one-hop
fat link V and a three-hop long (Naik) link W.  Links are passed with the
smearing and Naik coefficients already absorbed (the smearing that builds them
is not printed in the paper).  Readings:

* MILC phases (MILC order t, x, y, z): eta_t = 1, eta_x = (-1)^t,
  eta_y = (-1)^(t+x), eta_z = (-1)^(t+x+y).  The CPS order x, y, z, t used by
  Chroma gives eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z).
* D_MILC(m) chi = m chi + 1/2 sum_mu eta_mu(x) [V_mu(x) chi(x+mu)
      - V_mu^dag(x-mu) chi(x-mu) + W_mu(x) chi(x+3mu) - W_mu^dag(x-3mu) chi(x-3mu)],
  antiperiodic in time.  Chroma's operator carries the opposite mass sign:
  D_Chroma(m) = D_hop^CPS - m.  The sec. 2.2 field relation
  psi^Chroma = (-1)^{(t%2)((x+y+z)%2) + (x+y+z+t)%2} psi^QUDA then reads
  S D_MILC(m) S = -D_Chroma(m).
* Even-site normal operator: M_e(m) = m^2 - D_eo D_oe = (D^dag D)_ee.
"""
from __future__ import annotations

import numpy as np

from .lattice import coords, shift, parity, dims


def phases(L, convention="milc"):
    """eta_mu(x) for mu = 0..3 as a (4, Lt, Lz, Ly, Lx) array of +-1."""
    x, y, z, t = coords(L)
    one = np.ones_like(x)
    if convention == "milc":
        eta = [(-1) ** t, (-1) ** (t + x), (-1) ** (t + x + y), one]
    elif convention == "cps":
        eta = [one, (-1) ** x, (-1) ** (x + y), (-1) ** (x + y + z)]
    else:
        raise ValueError(convention)
    return np.array(eta, dtype=np.float64)


def chroma_sign(L):
    """S(x) = (-1)^{(t%2)((x+y+z)%2) + (x+y+z+t)%2} of the sec. 2.2 relation."""
    x, y, z, t = coords(L)
    return ((-1.0) ** ((t % 2) * ((x + y + z) % 2) + (x + y + z + t) % 2))


def _mv(U, v):
    return np.einsum("...ab,...b->...a", U, v)


def _mvd(U, v):
    return np.einsum("...ba,...b->...a", U.conj(), v)


def hop(V, W, chi, antiperiodic=True, convention="milc"):
    """1/2 sum_mu eta_mu [V chi(x+mu) - V^dag(x-mu) chi(x-mu) + W chi(x+3mu) - W^dag(x-3mu) chi(x-3mu)]."""
    L = dims(V.shape)
    eta = phases(L, convention)
    out = np.zeros_like(chi)
    for mu in range(4):
        Vm, Wm = V[..., mu, :, :], W[..., mu, :, :]
        s = _mv(Vm, shift(chi, mu, 1, antiperiodic))
        s -= _mvd(shift(Vm, mu, -1), shift(chi, mu, -1, antiperiodic))
        s += _mv(Wm, shift(chi, mu, 3, antiperiodic))
        s -= _mvd(shift(Wm, mu, -3), shift(chi, mu, -3, antiperiodic))
        out += eta[mu][..., None] * s
    return 0.5 * out


def hisq(V, W, chi, m, antiperiodic=True):
    """D_MILC(m) chi = m chi + D_hop chi."""
    return m * chi + hop(V, W, chi, antiperiodic)


def hisq_dag(V, W, chi, m, antiperiodic=True):
    """D^dag = m - D_hop (D_hop is anti-Hermitian)."""
    return m * chi - hop(V, W, chi, antiperiodic)


def chroma_op(V, W, chi, m, antiperiodic=True):
    """Chroma form with CPS phases and opposite mass sign: D_hop^CPS chi - m chi."""
    return hop(V, W, chi, antiperiodic, "cps") - m * chi


def even_mask(L):
    return (parity(L) == 0)[..., None]


def even_normal(V, W, chi_e, m, antiperiodic=True):
    """M_e(m) chi_e = m^2 chi_e - D_eo D_oe chi_e on even sites (zero elsewhere)."""
    L = dims(V.shape)
    ev = even_mask(L)
    chi_e = chi_e * ev
    t = hop(V, W, chi_e, antiperiodic) * (~ev)
    return (m * m * chi_e - hop(V, W, t, antiperiodic)) * ev
