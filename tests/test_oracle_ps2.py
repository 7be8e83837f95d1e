"""Pins for the oracle's two-site TDVP-PS step (oracle/ps2.py).

* merged MPO pair: replacing two MPO sites by their merged site leaves the
  dense Hamiltonian unchanged (brute force);
* full bond dimension: no truncation, every factor's projector pair sums
  as in the one-site scheme, so the step is exact: exp(-iHt) psi;
* truncated bond dimension: equal to the same two-site splitting applied
  literally to the dense state with dense projectors and dense truncated
  SVDs (oracle/dense.py, no environments, no merged MPO, no Krylov space);
* norm: the propagators are unitary, so the squared norm falls by exactly
  the weight each truncated SVD discards.
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw
from oracle import model, mps as om, ps2, dense


def test_merged_mpo_pair_gives_the_same_hamiltonian():
    p = draw_params(3, 1, 3, seed=2)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    ref = model.mpo_to_dense(Ws)
    for i in range(len(Ws) - 1):
        Wm = Ws[:i] + [ps2.merge_mpo(Ws[i], Ws[i + 1])] + Ws[i + 2:]
        assert np.abs(model.mpo_to_dense(Wm) - ref).max() < 1e-15 * max(np.abs(ref).max(), 1.0) * 10


def test_two_site_full_bond_is_exact():
    p = draw_params(2, 1, 3, seed=4)
    sites = chain_sites(p)
    H, _ = model.dense_hamiltonian(p, sites)
    Ws, _ = model.mpo(p, sites)
    m0 = om.right_canonicalize(initial_mps_raw(p, 6, 0.3, 2))
    T = 20 * model.AU_PER_FS
    ref = dense.exact_evolve(H, om.mps_to_dense(m0), [T])[0]
    m, _ = ps2.evolve2(m0, Ws, T / 10, 10)
    assert np.abs(om.mps_to_dense(m) - ref).max() < 1e-12


@pytest.mark.parametrize("n_e,n_modes,levels,M", [(3, 1, 4, 4), (3, 1, 4, 2), (2, 1, 3, 3)])
def test_two_site_truncated_equals_dense_projector_splitting(n_e, n_modes, levels, M):
    p = draw_params(n_e, n_modes, levels, seed=0)
    sites = chain_sites(p)
    H, _ = model.dense_hamiltonian(p, sites)
    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(initial_mps_raw(p, M, 1e-1, 1))
    dims = [A.shape[1] for A in m]
    bonds = [1] + [A.shape[2] for A in m]
    psi, phiL, phiR = dense.dense_projector_init(m)
    R = om.build_right_envs(m, Ws)
    tau = 2 * model.AU_PER_FS
    for _ in range(3):
        m, R, _ = ps2.ps2_step(m, Ws, R, tau)
        psi, phiL, phiR = dense.dense_projector_ps2_step(psi, phiL, phiR, H, dims, tau, bonds)
    assert np.abs(om.mps_to_dense(m) - psi).max() < 1e-12


def test_two_site_norm_falls_by_the_discarded_weight():
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(initial_mps_raw(p, 2, 1e-1, 1))
    R = om.build_right_envs(m, Ws)
    total = 0.0
    for _ in range(5):
        st = {}
        n0 = om.norm2(m)
        m, R, _ = ps2.ps2_step(m, Ws, R, 2 * model.AU_PER_FS, stats=st)
        assert sum(st["discarded"]) > 0.0
        assert abs(n0 - sum(st["discarded"]) - om.norm2(m)) < 1e-13
        total += sum(st["discarded"])
    assert abs(1.0 - total - om.norm2(m)) < 1e-12
