"""Pins for the oracle's Hamiltonian, MPO and units (Sec. II.C, eq:holstein, eq:mpo)."""

import numpy as np
import pytest
import scipy.constants as sc

from inputs import draw_params, chain_sites
from oracle import model


def test_unit_constants_match_codata():
    # 1 cm^-1 in hartree and 1 fs in atomic units of time, from scipy's CODATA tables
    hartree_per_m = sc.physical_constants["hartree-inverse meter relationship"][0]
    assert model.HARTREE_PER_CM == pytest.approx(100.0 / hartree_per_m, rel=1e-10)
    t_au = sc.physical_constants["atomic unit of time"][0]
    assert model.AU_PER_FS == pytest.approx(1e-15 / t_au, rel=1e-10)


@pytest.mark.parametrize("n_e,n_modes,levels", [(3, 1, 4), (2, 2, 3), (3, 0, 2), (4, 1, 2)])
def test_mpo_contracts_to_dense_hamiltonian(n_e, n_modes, levels):
    p = draw_params(n_e, n_modes, levels, seed=3)
    sites = chain_sites(p)
    H, shift = model.dense_hamiltonian(p, sites)
    Ws, shift2 = model.mpo(p, sites)
    Hm = model.mpo_to_dense(Ws)
    assert np.abs(H - H.conj().T).max() == 0.0
    assert np.abs(Hm - H).max() <= 1e-13 * np.abs(H).max()
    assert shift == shift2


def test_mpo_bond_dims_left_indexed():
    # 2 + 2k + [inside a vibrational block], k = electronic sites to the left
    p = draw_params(7, 10, 8, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    assert max(W.shape[0] for W in Ws) == 15
    assert Ws[0].shape[0] == 1 and Ws[-1].shape[3] == 1


def test_one_exciton_block_g0_is_textbook():
    # with g = 0 and no modes the one-exciton block is diag(E - Ebar) + J (in hartree)
    p = draw_params(4, 0, 2, seed=5)
    sites = chain_sites(p)
    H, shift = model.dense_hamiltonian(p, sites)
    n = len(sites)
    idx = []
    for s in sites:
        pos = [i for i, t in enumerate(sites) if t[1] == s[1]][0]
        idx.append(1 << (n - 1 - pos))   # site 0 is the most significant bit
    Hb = H[np.ix_(idx, idx)]
    E = p.E * model.HARTREE_PER_CM
    ref = np.diag(E - E.mean()) + p.J * model.HARTREE_PER_CM
    order = [s[1] for s in sites]
    ref = ref[np.ix_(order, order)]
    assert np.abs(Hb - ref).max() <= 1e-15
    assert shift == pytest.approx(E.mean())


def test_vibrational_block_spectrum():
    # a single electronic site with one mode: H' = w b+b + g w (b+ + b) n; with the
    # exciton present the displaced oscillator has levels w (k - g^2) (textbook),
    # up to truncation of the number basis
    p = draw_params(1, 1, 40, seed=2)
    sites = chain_sites(p)
    H, shift = model.dense_hamiltonian(p, sites)
    w = p.omega[0, 0] * model.HARTREE_PER_CM
    g2 = p.S[0, 0]
    lam = np.linalg.eigvalsh(H[40:, 40:])
    ref = w * (np.arange(5) - g2)
    assert np.abs(lam[:5] - ref).max() <= 1e-12 * w
