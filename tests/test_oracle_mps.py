"""Pins for the oracle's MPS primitives (eq:QR, eq:tdvp1_h, eq:tdvp1_H, eq:tdvp2_D).

Every local operator is checked against the dense Hamiltonian projected with
dense isometries, on tiny chains where that is cheap.
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw, random_complex
from oracle import model, mps as om, dense


@pytest.fixture(scope="module")
def small_chain():
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    H, shift = model.dense_hamiltonian(p, sites)
    Ws, _ = model.mpo(p, sites)
    mps = om.right_canonicalize(initial_mps_raw(p, 4, 1e-1, 7))
    return p, sites, H, Ws, mps


def _left_canonical_prefix(mps, upto):
    """Move the centre from site 0 to site ``upto`` with QR; returns new list."""
    m = [A.copy() for A in mps]
    for i in range(upto):
        ml, d, mr = m[i].shape
        Q, R = om.qr_pos(m[i].reshape(ml * d, mr))
        m[i] = Q.reshape(ml, d, mr)
        m[i + 1] = np.einsum("kr,rtq->ktq", R, m[i + 1])
    return m


def test_qr_identities():
    A = random_complex((40, 12), 1)
    Q, R = om.qr_pos(A)
    assert np.abs(Q.conj().T @ Q - np.eye(12)).max() < 1e-14
    assert np.abs(Q @ R - A).max() < 1e-14
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.all(np.diag(R).real >= 0) and np.abs(np.diag(R).imag).max() == 0.0


def test_cholesky_qr_is_the_unique_positive_diagonal_qr():
    """Shifted Cholesky QR (three passes): orthonormal Q, A = Q R, R upper
    triangular with positive real diagonal -- for full-rank A that
    factorisation is unique, so it must equal the Householder one."""
    A = random_complex((40, 12), 2)
    Q, R = om.qr_cholesky3(A)
    assert np.abs(Q.conj().T @ Q - np.eye(12)).max() < 1e-14
    assert np.abs(Q @ R - A).max() < 1e-13
    assert np.abs(np.tril(R, -1)).max() < 1e-15
    assert np.all(np.diag(R).real > 0) and np.abs(np.diag(R).imag).max() < 1e-15
    Qh, Rh = om.qr_pos(A)
    assert np.abs(Q - Qh).max() < 1e-13 and np.abs(R - Rh).max() < 1e-13


def test_cholesky_qr_ill_conditioned():
    """Singular values down to 1e-12 |A| (condition far beyond 1/sqrt(u)):
    still orthonormal to round-off and backward stable; the leading
    columns (well separated from the tiny singular values) agree with
    Householder."""
    U, _ = np.linalg.qr(random_complex((60, 16), 4))
    V, _ = np.linalg.qr(random_complex((16, 16), 5))
    A = (U * np.logspace(0, -12, 16)[None, :]) @ V.conj().T
    Q, R = om.qr_cholesky3(A)
    assert np.abs(Q.conj().T @ Q - np.eye(16)).max() < 1e-13
    assert np.abs(Q @ R - A).max() < 1e-14
    Qh, _ = om.qr_pos(A)
    assert np.abs(Q[:, 0] - Qh[:, 0]).max() < 1e-12


def test_right_canonical_condition(small_chain):
    _, _, _, _, mps = small_chain
    for A in mps[1:]:
        ml, d, mr = A.shape
        X = A.reshape(ml, d * mr)
        assert np.abs(X @ X.conj().T - np.eye(ml)).max() < 1e-13   # eq:rcanon
    assert om.norm2(mps) == pytest.approx(1.0, abs=1e-14)


def test_energy_from_environments_equals_dense(small_chain):
    _, _, H, Ws, mps = small_chain
    psi = om.mps_to_dense(mps)
    e_dense = np.vdot(psi, H @ psi)
    R = om.build_right_envs(mps, Ws)
    # <C0| H[0] |C0> with L[0] = 1 and R[1] from the right-canonical sites
    y = om.heff(om.ones_env(), Ws[0], R[1], mps[0])
    assert np.vdot(mps[0], y) == pytest.approx(e_dense, abs=1e-15)
    assert om.expectation_mpo(mps, Ws) == pytest.approx(e_dense, abs=1e-15)


@pytest.mark.parametrize("site", [0, 2, 3, 5])
def test_heff_equals_projected_dense(small_chain, site):
    _, _, H, Ws, mps = small_chain
    m = _left_canonical_prefix(mps, site)
    L = om.build_left_envs(m, Ws)
    R = om.build_right_envs(m, Ws)
    phiL = dense._left_iso(m[:site])
    phiR = dense._right_iso(m[site + 1:])
    d = m[site].shape[1]
    B = np.kron(np.kron(phiL, np.eye(d)), phiR.T)
    x = random_complex(m[site].shape, 11 + site)
    y = om.heff(L[site], Ws[site], R[site + 1], x)
    ref = (B.conj().T @ H @ B @ x.reshape(-1)).reshape(x.shape)
    assert np.abs(y - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("bond", [1, 3, 5])
def test_bond_operator_equals_projected_dense(small_chain, bond):
    _, _, H, Ws, mps = small_chain
    m = _left_canonical_prefix(mps, bond)
    L = om.build_left_envs(m, Ws)
    R = om.build_right_envs(m, Ws)
    phiL = dense._left_iso(m[:bond])
    phiR = dense._right_iso(m[bond:])
    B = np.kron(phiL, phiR.T)
    D = random_complex((phiL.shape[1], phiR.shape[0]), 21 + bond)
    y = om.bond_op(L[bond], R[bond], D)
    ref = (B.conj().T @ H @ B @ D.reshape(-1)).reshape(D.shape)
    assert np.abs(y - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_env_update_left_and_right_consistent(small_chain):
    # <psi|H|psi> from L[b] and R[b] at every bond (eq:tdvp1_h1i / eq:tdvp1_hiN)
    _, _, H, Ws, mps = small_chain
    psi = om.mps_to_dense(mps)
    e = np.vdot(psi, H @ psi)
    for b in range(1, len(mps)):
        m = _left_canonical_prefix(mps, b)
        L = om.build_left_envs(m, Ws)
        R = om.build_right_envs(m, Ws)
        # C at site b; energy = <C|H[b]|C>
        y = om.heff(L[b], Ws[b], R[b + 1], m[b])
        assert np.vdot(m[b], y) == pytest.approx(e, abs=1e-15)


def test_populations_equal_dense(small_chain):
    p, sites, H, Ws, mps = small_chain
    psi = om.mps_to_dense(mps)
    dims = [s[3] for s in sites]
    pops = om.site_populations(mps, sites, p.n_e)
    P = np.abs(psi.reshape(dims)) ** 2
    for pos, s in enumerate(sites):
        if s[0] == "el":
            ref = P.take(1, axis=pos).sum()
            assert pops[s[1]] == pytest.approx(ref, abs=1e-15)


def test_single_elements_match_brute_force_sums():
    """heff_element / env_left_element / env_right_element against the defining sums written
    out as loops over every index (tiny shapes), and against the full
    applications at a few points."""
    Ml, d, Mr, Wl, Wr = 3, 2, 2, 2, 3
    L = random_complex((Ml, Wl, Ml), 1)
    W = random_complex((Wl, d, d, Wr), 2)
    R = random_complex((Mr, Wr, Mr), 3)
    x = random_complex((Ml, d, Mr), 4)
    for (b, s, q) in [(0, 0, 0), (2, 1, 1), (1, 0, 1)]:
        ref = 0j
        for w in range(Wl):
            for k in range(Ml):
                for t in range(d):
                    for v in range(Wr):
                        for r in range(Mr):
                            ref += L[b, w, k] * W[w, s, t, v] * R[q, v, r] * x[k, t, r]
        assert abs(om.heff_element(L, W, R, x, b, s, q) - ref) < 1e-13
        assert abs(om.heff(L, W, R, x)[b, s, q] - ref) < 1e-13
    A = random_complex((Ml, d, Mr), 5)
    Wa = random_complex((Wl, d, d, Wr), 6)
    for (q, y, r) in [(0, 0, 0), (1, 2, 1), (0, 1, 1)]:
        ref = 0j
        for b in range(Ml):
            for w in range(Wl):
                for k in range(Ml):
                    for t in range(d):
                        for s in range(d):
                            ref += L[b, w, k] * A[k, t, r] * Wa[w, s, t, y] * np.conj(A[b, s, q])
        assert abs(om.env_left_element(L, A, Wa, q, y, r) - ref) < 1e-13
        assert abs(om.env_left(L, A, Wa)[q, y, r] - ref) < 1e-13
    Rr = random_complex((Mr, Wr, Mr), 7)
    for (b, w, k) in [(0, 0, 0), (2, 1, 1), (1, 1, 2)]:
        ref = 0j
        for q in range(Mr):
            for y in range(Wr):
                for r in range(Mr):
                    for t in range(d):
                        for s in range(d):
                            ref += Rr[q, y, r] * A[k, t, r] * Wa[w, s, t, y] * np.conj(A[b, s, q])
        assert abs(om.env_right_element(Rr, A, Wa, b, w, k) - ref) < 1e-13
        assert abs(om.env_right(Rr, A, Wa)[b, w, k] - ref) < 1e-13
