"""Lanczos approximation of y = exp(z A) x for Hermitian A (Sec. II.A.2, TDVP-PS).

The local equations eq:tdvp2_C and eq:tdvp2_D are linear, so each factor of
the splitting is a matrix exponential applied to a vector.  The paper builds
a Krylov space with the Lanczos three-term recurrence, diagonalises the
tridiagonal projected Hamiltonian T, and grows the space until the result
converges.  Here:

  v_0 = x / |x|
  w   = A v_j - beta_{j-1} v_{j-1};  alpha_j = Re <v_j, w>;  w -= alpha_j v_j
  w  -= V V^H w           (full classical Gram-Schmidt against v_0..v_j)
  beta_j = |w|;  v_{j+1} = w / beta_j

stopping at k = min(kmax, dim), at breakdown beta_j <= ``breakdown`` * |A v_j|
(the new direction is round-off of the applied vector; the paper does not
say how breakdown is detected, this relative test is the reading used), or
(if tol > 0) when the a-posteriori estimate |z beta_j [exp(z T_k) e_1]_k|
drops below tol.  Then T_k = Q diag(lam) Q^T (numpy.linalg.eigh) and
y = |x| V_k Q exp(z lam) Q^T e_1.
"""

from __future__ import annotations

import numpy as np


def exp_tridiag_e1(alpha, beta, z):
    """exp(z T) e_1 for the real symmetric tridiagonal T(alpha, beta)."""
    k = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=float))
    if k > 1:
        off = np.asarray(beta[: k - 1], dtype=float)
        T += np.diag(off, 1) + np.diag(off, -1)
    lam, Q = np.linalg.eigh(T)
    return Q @ (np.exp(z * lam) * Q[0, :])


def expm_lanczos(apply, x, z, kmax=20, tol=0.0, breakdown=1e-12, info=None):
    """Return exp(z A) x with A given by ``apply`` (same shape in and out)."""
    shape = x.shape
    xv = np.asarray(x, dtype=np.complex128).reshape(-1)
    nrm = np.linalg.norm(xv)
    if nrm == 0.0:
        if info is not None:
            info["k"] = 0
        return np.zeros(shape, dtype=np.complex128)
    kmax = max(1, min(kmax, xv.size))
    V = [xv / nrm]
    alpha, beta = [], []
    k = 0
    for j in range(kmax):
        w = apply(V[j].reshape(shape)).reshape(-1).astype(np.complex128)
        aw = float(np.linalg.norm(w))
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        a = float(np.vdot(V[j], w).real)
        w = w - a * V[j]
        Vm = np.array(V)
        w = w - Vm.T @ (Vm.conj() @ w)
        alpha.append(a)
        b = float(np.linalg.norm(w))
        k = j + 1
        if k == kmax or b <= breakdown * aw:
            break
        if tol > 0.0:
            c = exp_tridiag_e1(alpha, beta, z)
            if abs(z * b * c[-1]) < tol:
                break
        beta.append(b)
        V.append(w / b)
    c = exp_tridiag_e1(alpha, beta, z)
    y = nrm * (np.array(V[:k]).T @ c)
    if info is not None:
        info["k"] = k
    return y.reshape(shape)
