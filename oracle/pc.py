"""Propagation and compression with RK4 (P&C-RK4, Sec. II.A.1, eq:RK4),
built from the MPS operations of Sec. II.A: MPO x MPS (eq:mpo-apply),
MPS + MPS (eq:mps+mps), canonicalisation by QR (eq:QR) and compression by
truncated SVD (eq:SVD).

Test infrastructure: a plain FP64 reference, sharing no code with the GPU
path (which does not implement this scheme yet).

One step of size tau for the time-independent H (eq:RK4 with H(t) = H):
  k1 = -i H psi,  k2 = -i H (psi + tau/2 k1),  k3 = -i H (psi + tau/2 k2),
  k4 = -i H (psi + tau k3),  psi' = psi + tau/6 (k1 + 2 k2 + 2 k3 + k4);
every product and every sum is compressed to the target bond dimensions
right after it is formed (the paper compresses after each operation): the
raw MPS is left-canonicalised by a QR sweep and then compressed by a
truncated-SVD sweep from the last site to the first (largest singular
values kept, fixed bond dimension per bond), which leaves it right
canonical with the norm on site 0.

Pins (tests): MPO x MPS and MPS + MPS against the dense operations;
compression exact when the bond dimensions hold the state's Schmidt ranks;
at full bond dimension one step equals the fourth-order Taylor polynomial
of exp(-i H tau) applied to psi (what RK4 computes for a linear,
time-independent equation), and the error against exp(-i H t) falls at
fourth order in tau.
"""

from __future__ import annotations

import numpy as np

from .mps import qr_pos


def mpo_apply(Ws, mps):
    """eq:mpo-apply: A'[(w a), s, (v b)] = sum_t W[w, s, t, v] A[a, t, b]."""
    out = []
    for W, A in zip(Ws, mps):
        wl, d, _, wr = W.shape
        ml, _, mr = A.shape
        T = np.einsum("wstv,atb->wasvb", W, A)
        out.append(T.reshape(wl * ml, d, wr * mr))
    return out


def mps_add(a, b):
    """eq:mps+mps: block-diagonal merge (first site side by side, last site stacked)."""
    n = len(a)
    if n == 1:
        return [a[0] + b[0]]
    out = []
    for i, (A, B) in enumerate(zip(a, b)):
        la, d, ra = A.shape
        lb, _, rb = B.shape
        if i == 0:
            out.append(np.concatenate([A, B], axis=2))
        elif i == n - 1:
            out.append(np.concatenate([A, B], axis=0))
        else:
            C = np.zeros((la + lb, d, ra + rb), dtype=np.complex128)
            C[:la, :, :ra] = A
            C[la:, :, ra:] = B
            out.append(C)
    return out


def scale(mps, c):
    out = [A.copy() for A in mps]
    out[0] = out[0] * c
    return out


def compress(mps, bonds):
    """QR sweep left to right (eq:QR), then truncated-SVD sweep right to left
    (eq:SVD) keeping bonds[b] singular values at bond b (b = 1 .. N-1)."""
    m = [A.astype(np.complex128).copy() for A in mps]
    n = len(m)
    for i in range(n - 1):
        ml, d, mr = m[i].shape
        Q, R = qr_pos(m[i].reshape(ml * d, mr))
        k = Q.shape[1]
        m[i] = Q.reshape(ml, d, k)
        m[i + 1] = np.einsum("kr,rtq->ktq", R, m[i + 1])
    for i in range(n - 1, 0, -1):
        ml, d, mr = m[i].shape
        U, S, Vh = np.linalg.svd(m[i].reshape(ml, d * mr), full_matrices=False)
        k = min(bonds[i], S.size)
        m[i] = Vh[:k].reshape(k, d, mr)
        m[i - 1] = np.einsum("lsk,kr->lsr", m[i - 1], U[:, :k] * S[:k])
    return m


def pc_rk4_step(mps, Ws, tau, bonds):
    """One P&C-RK4 step (eq:RK4) with compression to `bonds` after every operation."""
    def H(x):
        return compress(scale(mpo_apply(Ws, x), -1j), bonds)

    def add(x, y, c):
        return compress(mps_add(x, scale(y, c)), bonds)

    k1 = H(mps)
    k2 = H(add(mps, k1, 0.5 * tau))
    k3 = H(add(mps, k2, 0.5 * tau))
    k4 = H(add(mps, k3, tau))
    out = add(mps, k1, tau / 6)
    out = add(out, k2, tau / 3)
    out = add(out, k3, tau / 3)
    return add(out, k4, tau / 6)


def pc_rk4_evolve(mps, Ws, tau, nsteps, bonds):
    m = [A.astype(np.complex128) for A in mps]
    for _ in range(nsteps):
        m = pc_rk4_step(m, Ws, tau, bonds)
    return m
