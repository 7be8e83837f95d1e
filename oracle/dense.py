"""Dense references for tiny chains.

* :func:`exact_evolve` -- psi(t) = exp(-i H t) psi(0) through numpy.linalg.eigh.
* :func:`dense_projector_ps_step` -- the same symmetric splitting as the PS
  step (eq:ps_trotter), but every factor is applied literally to the dense
  state as psi <- expm(-+ i h P H P) psi with the dense projector
  P = (Phi_L Phi_L^H) (x) I_i (x) (Phi_R^T Phi_R^*) built from dense
  isometries.  The centre move is implicit (the next local tensor is read
  off psi), and there are no environments and no Krylov space, so this pins
  the MPS step at truncated bond dimension through code it does not share.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from .mps import qr_pos


def exact_evolve(H, psi0, times):
    lam, V = np.linalg.eigh(H)
    c = V.conj().T @ psi0
    return [V @ (np.exp(-1j * lam * t) * c) for t in times]


def _left_iso(mps_left):
    """Dense left isometry (D_left x M) from left-canonical tensors."""
    P = np.ones((1, 1), dtype=np.complex128)
    for A in mps_left:
        P = np.einsum("pk,ksr->psr", P, A).reshape(-1, A.shape[2])
    return P


def _right_iso(mps_right):
    """Dense right isometry (M x D_right), orthonormal rows."""
    P = np.ones((1, 1), dtype=np.complex128)
    for A in reversed(mps_right):
        P = np.einsum("ksr,rq->ksq", A, P).reshape(A.shape[0], -1)
    return P


def _apply_factor(psi, H, B, z):
    """psi <- expm(z P H P) psi with P = B B^H (dense)."""
    P = B @ B.conj().T
    return scipy.linalg.expm(z * (P @ H @ P)) @ psi


def dense_projector_ps_step(psi, phiL, phiR, H, dims, tau):
    """One symmetric step in dense form.

    ``phiL[b]`` is the dense left isometry of sites 0..b-1 (D_left x M_b),
    ``phiR[b]`` the dense right isometry of sites b..N-1 (M_b x D_right);
    on entry phiR[1..N] describe the right-canonical state, phiL[0] = [[1]].
    Returns the new psi and updated isometry lists.
    """
    n = len(dims)
    phiL = list(phiL)
    phiR = list(phiR)
    h = 0.5 * tau
    one = np.ones((1, 1), dtype=np.complex128)
    phiL[0] = one
    phiR[n] = one

    def site_basis(i):
        return np.kron(np.kron(phiL[i], np.eye(dims[i])), phiR[i + 1].T)

    def bond_basis(b):
        return np.kron(phiL[b], phiR[b].T)

    for i in range(n):
        last = i == n - 1
        B = site_basis(i)
        psi = _apply_factor(psi, H, B, -1j * (tau if last else h))
        if last:
            break
        C = B.conj().T @ psi
        ml, mr = phiL[i].shape[1], phiR[i + 1].shape[0]
        Q, _ = qr_pos(C.reshape(ml * dims[i], mr))
        phiL[i + 1] = np.kron(phiL[i], np.eye(dims[i])) @ Q
        psi = _apply_factor(psi, H, bond_basis(i + 1), 1j * h)
    for i in range(n - 1, -1, -1):
        B = site_basis(i)
        if i < n - 1:
            psi = _apply_factor(psi, H, B, -1j * h)
        if i == 0:
            break
        C = B.conj().T @ psi
        ml, mr = phiL[i].shape[1], phiR[i + 1].shape[0]
        Q, _ = qr_pos(C.reshape(ml, dims[i] * mr).conj().T)
        phiR[i] = Q.conj().T @ np.kron(np.eye(dims[i]), phiR[i + 1])
        psi = _apply_factor(psi, H, bond_basis(i), 1j * h)
    return psi, phiL, phiR


def dense_projector_init(mps_rc):
    """Dense isometries and state from a right-canonical MPS (centre at site 0)."""
    n = len(mps_rc)
    phiR = [None] * (n + 1)
    for b in range(1, n + 1):
        phiR[b] = _right_iso(mps_rc[b:]) if b < n else np.ones((1, 1), dtype=np.complex128)
    phiL = [np.ones((1, 1), dtype=np.complex128)] + [None] * n
    psi = (mps_rc[0].reshape(-1, mps_rc[0].shape[2]) @ phiR[1]).reshape(-1)
    return psi, phiL, phiR


def dense_projector_ps2_step(psi, phiL, phiR, H, dims, tau, bonds):
    """One symmetric two-site step in dense form (the splitting of
    oracle.ps2.ps2_step): every forward factor is expm(-i h P2 H P2) on the
    dense state with the two-site projector of pair (i, i+1), every
    backward factor expm(+i h P1 H P1) with the one-site projector; each
    split reads the pair's coefficients off psi, keeps the bonds[i+1]
    largest singular values, replaces psi by the truncated state and
    extends the dense isometry by the kept singular vectors.  No
    environments, no merged MPO, no Krylov space."""
    n = len(dims)
    phiL = list(phiL)
    phiR = list(phiR)
    h = 0.5 * tau
    one = np.ones((1, 1), dtype=np.complex128)
    phiL[0] = one
    phiR[n] = one

    def pair_basis(i):
        return np.kron(np.kron(phiL[i], np.eye(dims[i] * dims[i + 1])), phiR[i + 2].T)

    def site_basis(i):
        return np.kron(np.kron(phiL[i], np.eye(dims[i])), phiR[i + 1].T)

    def split(i, B, left_iso):
        ml, mr = phiL[i].shape[1], phiR[i + 2].shape[0]
        X = (B.conj().T @ psi).reshape(ml * dims[i], dims[i + 1] * mr)
        U, S, Vh = np.linalg.svd(X, full_matrices=False)
        m = bonds[i + 1]
        U, S, Vh = U[:, :m], S[:m], Vh[:m]
        new_psi = B @ ((U * S) @ Vh).reshape(-1)
        if left_iso:
            phiL[i + 1] = np.kron(phiL[i], np.eye(dims[i])) @ U
        else:
            phiR[i + 1] = Vh @ np.kron(np.eye(dims[i + 1]), phiR[i + 2])
        return new_psi

    for i in range(n - 1):
        last = i == n - 2
        B = pair_basis(i)
        psi = _apply_factor(psi, H, B, -1j * (tau if last else h))
        psi = split(i, B, left_iso=not last)
        if last:
            break
        psi = _apply_factor(psi, H, site_basis(i + 1), 1j * h)
    for i in range(n - 3, -1, -1):
        psi = _apply_factor(psi, H, site_basis(i + 1), 1j * h)
        B = pair_basis(i)
        psi = _apply_factor(psi, H, B, -1j * h)
        psi = split(i, B, left_iso=False)
    return psi, phiL, phiR
