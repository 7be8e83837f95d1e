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


def _mu_state_with_tiny_singular_value(lam_small):
    """Left-canonical 6-site state (bond dims 1,2,4,4,4,4,1; bonds 2-4
    truncated) whose Schmidt values at bond 4 are (0.9, 0.4, 0.1,
    lam_small) up to normalisation: the last two site tensors come from a
    QR of X = U diag(lam) V^H, X the (M_4, d_4 d_5) matrix of the state to
    the right of bond 4.  Returns the site index i = 3 whose bond matrix
    D_i (bond 4) carries the small singular value."""
    from inputs import random_complex
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    m = mu.left_canonicalize(initial_mps_raw(p, 4, 1e-1, 1))
    M4, d4, _ = m[4].shape
    d5 = m[5].shape[1]
    U, _ = np.linalg.qr(random_complex((M4, M4), 31))
    V, _ = np.linalg.qr(random_complex((d4 * d5, M4), 32))
    lam = np.array([0.9, 0.4, 0.1, lam_small])
    lam = lam / np.linalg.norm(lam)
    X = U @ np.diag(lam) @ V.conj().T                       # M4 x (d4 d5)
    Q, R = np.linalg.qr(X.reshape(M4 * d4, d5))
    m[4] = Q.reshape(M4, d4, d5)
    m[5] = R.reshape(d5, d5, 1)
    return p, sites, Ws, m, 3


def _dense_mu_site_derivative(p, sites, m, i, eps):
    """eq:tdvp1_mu_L for site i, evaluated with dense matrices and written
    independently of oracle/mu.py: dense H, the dense left isometries of
    sites 0..i-1 and 0..i, an orthonormal basis of the row space of the
    state right of bond i+1 (QR of the dense contraction of the sites to
    the right), and the regularised inverse of eq:reg2."""
    H, _ = model.dense_hamiltonian(p, sites)
    psi = om.mps_to_dense(m)
    Phi = np.ones((1, 1), complex)
    for A in m[:i]:
        Phi = np.einsum("pk,ksr->psr", Phi, A).reshape(-1, A.shape[2])
    ml, d, mr = m[i].shape
    Phi_i = np.einsum("pk,ksr->psr", Phi, m[i]).reshape(-1, mr)
    # Y: (M_{i+1}) x (right dims), the state right of bond i+1 (psi = Phi_i Y)
    Y = m[i + 1].reshape(mr, -1)
    for A in m[i + 2:]:
        Y = np.einsum("bqp,psr->bqsr", Y.reshape(mr, -1, A.shape[0]), A).reshape(mr, -1)
    dR = Y.shape[1]
    Q, _ = np.linalg.qr(Y.conj().T)                 # dR x mr, orthonormal, spans Y's rows
    Psi = psi.reshape(-1, dR)
    D = Phi_i.conj().T @ Psi @ Q                    # bond matrix in the basis Phi_i x Q
    Hpsi = (H @ psi).reshape(Phi.shape[0], d, dR)
    G = np.einsum("pl,psr->lsr", Phi.conj(), Hpsi @ Q).reshape(ml * d, mr)
    U, lam, Vh = np.linalg.svd(D)
    lam_t = lam + np.sqrt(eps) * np.exp(-lam / np.sqrt(eps))
    X = G @ Vh.conj().T @ np.diag(1.0 / lam_t) @ U.conj().T
    Am = m[i].reshape(ml * d, mr)
    X = X - Am @ (Am.conj().T @ X)
    return -1j * X, U, lam


@pytest.mark.parametrize("lam_small,eps", [(9e-6, 1e-10), (1e-6, 1e-10), (1e-7, 1e-12), (1e-8, 1e-10)])
def test_mu_rhs_regulariser_matches_dense_evaluation(lam_small, eps):
    """Pin of eq:reg2: with a bond singular value lam at, below or far below
    sqrt(eps), mu_rhs equals a dense evaluation of eq:tdvp1_mu_L with the
    regularised inverse (a mistaken eps for sqrt(eps), or a regularised
    Lambda^2, changes the result by orders of magnitude there).  The
    tolerance follows the conditioning of the data: the singular direction
    of lam is fixed by the tensors only to ~1e-16 / lam, and the
    regulariser amplifies that direction by 1/sqrt(eps)."""
    p, sites, Ws, m, i = _mu_state_with_tiny_singular_value(lam_small)
    ref, _, lam = _dense_mu_site_derivative(p, sites, m, i, eps)
    assert lam.min() <= np.sqrt(eps) * 1.001
    got = mu.mu_rhs(m, Ws, eps)[i].reshape(ref.shape)
    assert np.abs(got - ref).max() < (1e-15 / lam.min()) * np.abs(ref).max()


def test_mu_rhs_regularised_direction_scales_as_inverse_sqrt_eps():
    """For a singular value lam far below sqrt(eps), the regularised inverse
    is ~1/sqrt(eps): the part of dL/dt along that singular direction grows
    tenfold when eps drops a hundredfold, while the parts along the large
    singular values do not change (a closed-form consequence of eq:reg2)."""
    p, sites, Ws, m, i = _mu_state_with_tiny_singular_value(1e-8)
    _, U, lam = _dense_mu_site_derivative(p, sites, m, i, 1e-10)
    k = int(np.argmin(lam))
    big = int(np.argmax(lam))
    a = mu.mu_rhs(m, Ws, 1e-10)[i]
    b = mu.mu_rhs(m, Ws, 1e-12)[i]
    ml, d, mr = a.shape
    a, b = a.reshape(ml * d, mr), b.reshape(ml * d, mr)
    ratio = np.linalg.norm(b @ U[:, k]) / np.linalg.norm(a @ U[:, k])
    assert ratio == pytest.approx(10.0, rel=1e-3)
    assert np.linalg.norm(b @ U[:, big]) == pytest.approx(np.linalg.norm(a @ U[:, big]), rel=1e-9)


# --- constant mean field, second order (midpoint) --------------------------

def _cmf_case():
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    m0 = mu.left_canonicalize(initial_mps_raw(p, 4, 1e-1, 1))
    return p, sites, Ws, m0


def test_cmf_is_second_order_in_tau():
    """At truncated bond dimension the CMF steps converge to the solution of
    the same equations of motion integrated with live mean fields (VMF,
    tight tolerance) at second order in tau, as the paper reports for its
    CMF runs (error slope 2 against tau).  The same schedule with the mean
    fields of the step's start state held over the whole step (a first-order
    scheme) converges at first order only, so the test tells the midpoint
    fields from a mistaken freeze."""
    _, _, Ws, m0 = _cmf_case()
    T = 10 * model.AU_PER_FS
    mf, _, _ = mu.mu_evolve(m0, Ws, T, eps=1e-10, rtol=1e-11, atol=1e-13)
    ref = om.mps_to_dense(mf)
    errs, errs1 = [], []
    for nst in (10, 20, 40):
        m = mu.mu_cmf_evolve(m0, Ws, T / nst, nst, rtol=1e-11, atol=1e-13)
        errs.append(np.abs(om.mps_to_dense(m) - ref).max())
        m1 = [A.copy() for A in m0]
        for _ in range(nst):
            m1 = mu.cmf_propagate(m1, Ws, mu.mu_fields(m1, Ws), T / nst, 1e-11, 1e-13)
        errs1.append(np.abs(om.mps_to_dense(m1) - ref).max())
    assert errs[-1] < 2e-5
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.6
    for a, b in zip(errs1, errs1[1:]):
        assert 1.6 < a / b < 2.4


def test_cmf_full_bond_converges_to_exact():
    """Full bond dimension, full Schmidt rank: the equations of motion are
    exact, so CMF converges to exp(-iHt) psi(0) at second order."""
    p = draw_params(2, 1, 3, seed=4)
    sites = chain_sites(p)
    H, _ = model.dense_hamiltonian(p, sites)
    Ws, _ = model.mpo(p, sites)
    m0 = mu.left_canonicalize(initial_mps_raw(p, 6, 0.3, 2))
    T = 10 * model.AU_PER_FS
    ref = dense.exact_evolve(H, om.mps_to_dense(m0), [T])[0]
    errs = []
    for nst in (10, 20, 40):
        m = mu.mu_cmf_evolve(m0, Ws, T / nst, nst, eps=1e-14, rtol=1e-11, atol=1e-13)
        errs.append(np.abs(om.mps_to_dense(m) - ref).max())
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.6


def test_cmf_keeps_norm_and_gauge():
    """The centre's propagator is unitary and each L_i's frozen-field
    equation keeps L_i^H L_i constant, so both survive to the integrator's
    tolerance."""
    _, _, Ws, m0 = _cmf_case()
    m = mu.mu_cmf_evolve(m0, Ws, 2 * model.AU_PER_FS, 3, rtol=1e-11, atol=1e-13)
    assert abs(np.linalg.norm(om.mps_to_dense(m)) - 1.0) < 1e-10
    for A in m[:-1]:
        ml, d, mr = A.shape
        X = A.reshape(ml * d, mr)
        assert np.abs(X.conj().T @ X - np.eye(mr)).max() < 1e-9
