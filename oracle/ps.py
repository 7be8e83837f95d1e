"""One symmetric TDVP-PS time step (eq:ps_trotter, eq:tdvp2_C, eq:tdvp2_D).

Entry state: right-canonical MPS with the gauge centre C at site 0 and every
right environment R[1..N] built from it.  One step of size tau is a
left-to-right sweep then a right-to-left sweep, each with h = tau/2:

  LR, site i = 0..N-1:  C_i <- exp(-i h H[i]) C_i            (forward, eq:tdvp2_C)
                         C_i = L_i D  (QR, eq:QR)             (i < N-1)
                         L[i+1] <- env_left(L[i], L_i, W_i)
                         D <- exp(+i h K_{i+1}) D              (backward, eq:tdvp2_D)
                         C_{i+1} <- D R_{i+1}                  (centre move)
  RL, site i = N-1..0:  mirror image with RQ, env_right and C_{i-1} = L_{i-1} D

The two forward factors on the last site use the same projector one after
the other, so they are merged into a single exp(-i tau H[N-1]).
Returns the new MPS (same gauge as on entry) and the updated environments.
qr is the thin QR of eq:QR: numpy's Householder QR by default; the
shifted Cholesky QR of oracle.mps.qr_cholesky3 gives a second,
equally valid run for measuring the trajectory's rounding sensitivity.
"""

from __future__ import annotations

import numpy as np

from .krylov import expm_lanczos
from .mps import qr_pos, env_left, env_right, heff, bond_op, ones_env, build_right_envs


def ps_step(mps, Ws, R, tau, kmax=20, tol=0.0, L=None, stats=None, qr=qr_pos):
    n = len(mps)
    mps = [A.copy() for A in mps]
    R = list(R)
    if L is None:
        L = [None] * (n + 1)
    L = list(L)
    L[0] = ones_env()
    R[n] = ones_env()
    h = 0.5 * tau
    ks = []

    def fwd(i, z):
        info = {}
        out = expm_lanczos(lambda x: heff(L[i], Ws[i], R[i + 1], x), mps[i], z,
                           kmax=kmax, tol=tol, info=info)
        ks.append(info["k"])
        return out

    def bwd(b, D, z):
        info = {}
        out = expm_lanczos(lambda x: bond_op(L[b], R[b], x), D, z,
                           kmax=kmax, tol=tol, info=info)
        ks.append(info["k"])
        return out

    # left-to-right half sweep
    for i in range(n):
        last = i == n - 1
        mps[i] = fwd(i, -1j * (tau if last else h))
        if last:
            break
        ml, d, mr = mps[i].shape
        Q, D = qr(mps[i].reshape(ml * d, mr))
        mps[i] = Q.reshape(ml, d, mr)
        L[i + 1] = env_left(L[i], mps[i], Ws[i])
        D = bwd(i + 1, D, 1j * h)
        mps[i + 1] = np.einsum("kr,rtq->ktq", D, mps[i + 1])
    # right-to-left half sweep
    for i in range(n - 1, -1, -1):
        if i < n - 1:
            mps[i] = fwd(i, -1j * h)
        if i == 0:
            break
        ml, d, mr = mps[i].shape
        Q, Rf = qr(mps[i].reshape(ml, d * mr).conj().T)
        mps[i] = Q.conj().T.reshape(ml, d, mr)
        D = Rf.conj().T
        R[i] = env_right(R[i + 1], mps[i], Ws[i])
        D = bwd(i, D, 1j * h)
        mps[i - 1] = np.einsum("lsk,kr->lsr", mps[i - 1], D)
    if stats is not None:
        stats["k"] = ks
    return mps, R, L


def evolve(mps, Ws, tau, nsteps, kmax=20, tol=0.0, observe=None):
    """Run nsteps PS steps from a right-canonical MPS; call observe(t, mps) each step."""
    R = build_right_envs(mps, Ws)
    out = []
    if observe is not None:
        out.append(observe(0.0, mps))
    for s in range(nsteps):
        mps, R, _ = ps_step(mps, Ws, R, tau, kmax=kmax, tol=tol)
        if observe is not None:
            out.append(observe((s + 1) * tau, mps))
    return mps, out
