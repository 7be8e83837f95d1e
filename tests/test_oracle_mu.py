"""Pins for the TDVP-MU oracle (eq:tdvp1_C, eq:tdvp1_mu_L, eq:reg2).

* Full bond dimension with full Schmidt rank: the TDVP equations are exact,
  so MU (tight RK45, small eps) must equal exp(-iHt) psi(0).
* Truncated bond dimension: the paper states that MU and PS give the same
  state at converged step size (qualitative; parity unpinned).  Measured
  here: the PS result converges to the MU result at second order in tau.
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw
from oracle import model, mps as om, mu, ps, dense


def test_mu_full_rank_full_bond_is_exact():
    p = draw_params(2, 1, 3, seed=4)
    sites = chain_sites(p)
    H, _ = model.dense_hamiltonian(p, sites)
    Ws, _ = model.mpo(p, sites)
    m0 = mu.left_canonicalize(initial_mps_raw(p, 6, 0.3, 2))
    psi0 = om.mps_to_dense(m0)
    T = 20 * model.AU_PER_FS
    mf, _, _ = mu.mu_evolve(m0, Ws, T, eps=1e-14, rtol=1e-10, atol=1e-12)
    ref = dense.exact_evolve(H, psi0, [T])[0]
    assert np.abs(om.mps_to_dense(mf) - ref).max() < 1e-9


def test_mu_rhs_keeps_gauge_tangent():
    # L_i^H dL_i/dt = 0 (the derivative lies in the tangent space of the gauge)
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    m = mu.left_canonicalize(initial_mps_raw(p, 4, 1e-1, 1))
    d = mu.mu_rhs(m, Ws)
    for A, dA in zip(m[:-1], d[:-1]):
        ml, dd, mr = A.shape
        X = A.reshape(ml * dd, mr).conj().T @ dA.reshape(ml * dd, mr)
        assert np.abs(X).max() < 1e-13


@pytest.mark.slow
def test_ps_converges_to_mu_at_second_order():
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    raw = initial_mps_raw(p, 4, 1e-1, 1)
    mL = mu.left_canonicalize(raw)
    mR = om.right_canonicalize(raw)
    T = 10 * model.AU_PER_FS
    mf, _, _ = mu.mu_evolve(mL, Ws, T, eps=1e-12, rtol=1e-10, atol=1e-12)
    psi_mu = om.mps_to_dense(mf)
    errs = []
    for nst in (10, 40, 160):
        m, _ = ps.evolve(mR, Ws, T / nst, nst)
        errs.append(np.abs(om.mps_to_dense(m) - psi_mu).max())
    assert errs[2] < 1e-6
    for a, b in zip(errs, errs[1:]):
        assert 10.0 < a / b < 25.0     # 4x smaller step -> ~16x smaller difference
