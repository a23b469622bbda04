"""The per-site oracle (used for full-size GPU checks) equals the whole-lattice
oracle at every site of small lattices with ragged, unequal extents."""
import numpy as np
import pytest

import synth
from oracle import overlap as O
from oracle import sampled as SM
from oracle import staggered as S
from oracle import wilson as W
from oracle.lattice import parity

LATS = [(4, 4, 4, 6), (6, 4, 4, 8)]


def _all_sites(L, par=None):
    Lx, Ly, Lz, Lt = L
    return [(t, z, y, x) for t in range(Lt) for z in range(Lz) for y in range(Ly) for x in range(Lx)
            if par is None or (x + y + z + t) % 2 == par]


@pytest.mark.parametrize("L", LATS)
def test_tm_clover_and_hw_per_site(L):
    U = synth.su3_field(L, 0.4, 3)
    psi = synth.gaussian_spinor(L, 1, 4)[0]
    m, csw, mu = -0.3, 1.2, 0.07
    full = W.tm_clover(U, psi, m, csw, mu)
    wil = W.wilson(U, psi, m)
    hw = O.hw(U, psi, 1.5)
    for s in _all_sites(L)[::3]:
        assert np.allclose(SM.tm_clover_at(U, psi, m, csw, mu, s), full[s], atol=1e-12)
        assert np.allclose(SM.wilson_at(U, psi, m, s), wil[s], atol=1e-12)
        assert np.allclose(SM.hw_at(U, psi, 1.5, s), hw[s], atol=1e-12)


@pytest.mark.parametrize("L", LATS)
def test_schur_per_site(L):
    U = synth.su3_field(L, 0.4, 5)
    psi = synth.gaussian_spinor(L, 1, 6)[0]
    m, csw, mu = -0.2, 1.0509, 0.05
    eo = W.EvenOdd(U, m, csw, mu)
    ev = (parity(L) == 0)[..., None, None]
    full = eo.mhat(psi * ev)
    for s in _all_sites(L, 0)[::2]:
        assert np.allclose(SM.schur_at(U, psi * ev, m, csw, mu, s), full[s], atol=1e-12)


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (6, 4, 8, 6)])
def test_hisq_per_site(L):
    V, Wl = synth.hisq_fields(L, 7)
    chi = synth.gaussian_colour(L, 1, 8)[0]
    hop = S.hop(V, Wl, chi)
    ev = S.even_mask(L)
    ne = S.even_normal(V, Wl, chi * ev, 0.03)
    for s in _all_sites(L)[::3]:
        assert np.allclose(SM.stag_hop_at(V, Wl, chi, s), hop[s], atol=1e-12)
    for s in _all_sites(L, 0)[::2]:
        assert np.allclose(SM.even_normal_at(V, Wl, chi * ev, 0.03, s), ne[s], atol=1e-12)


def test_sample_sites():
    L = (6, 4, 8, 10)
    s = SM.sample_sites(L, 50, 1, parity=0)
    assert len(set(s)) == 50 and all(sum(x) % 2 == 0 for x in s)
    assert all(0 <= t < 10 and 0 <= z < 8 and 0 <= y < 4 and 0 <= x < 6 for t, z, y, x in s)
    assert s == SM.sample_sites(L, 50, 1, parity=0)
