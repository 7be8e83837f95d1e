"""Two-site TDVP-PS (the two-site form of the projector-splitting scheme
that Sec. II.A.2 mentions after eq:tdvp2_D, with an adaptive basis at each
bond and the cost the paper cites as its reason to use the one-site form).

Test infrastructure: a plain FP64 reference for the GPU path, sharing no
code with it.

The projector of eq:ps_trotter is split over neighbouring PAIRS of sites:
the forward factors act on the two-site tensor X_{i,i+1} = C_i A_{i+1}
with the two-site operator H[i,i+1] = h[1:i-1] W[i] W[i+1] h[i+2:N]
(eq:tdvp1_H with two MPO sites), the backward factors on the one-site
centre with H[i] (eq:tdvp2_C run backwards).  After each forward factor
the pair is split by an SVD truncated to the bond's dimension (eq:SVD,
the largest singular values kept), which chooses the bond basis anew: the
adaptive part of the scheme.  One step of size tau, h = tau/2:

  LR, pair i = 0..N-2:  X <- exp(-i h H[i,i+1]) X               (forward)
                        X = U S V^H, A_i = U, C_{i+1} = S V^H      (i < N-2)
                        L[i+1] <- env_left(L[i], A_i, W_i)
                        C_{i+1} <- exp(+i h H[i+1]) C_{i+1}        (backward)
  the last pair takes exp(-i tau H[N-2,N-1]) (its two forward factors
  meet), then splits with the centre on its left site, C_{N-2} = U S,
  B_{N-1} = V^H;
  RL, pair i = N-3..0:  C_{i+1} <- exp(+i h H[i+1]) C_{i+1}        (backward)
                        X = A_i C_{i+1}; X <- exp(-i h H[i,i+1]) X
                        X = U S V^H, C_i = U S, B_{i+1} = V^H
                        R[i+1] <- env_right(R[i+2], B_{i+1}, W_{i+1})

Bond dimensions are those of the entry state (fixed maximal M per bond);
no singular-value threshold.  Entry and exit gauge as in ps.ps_step: right
canonical, centre at site 0, right environments R[1..N] valid.

Pins (tests): exact at full bond dimension (no truncation) against
exp(-iHt) psi; at truncated bond dimension the discarded weight is the
only loss of norm (norm^2 + discarded weight = 1 per split); energy
conserved to the truncation; second-order convergence in tau.
"""

from __future__ import annotations

import numpy as np

from .krylov import expm_lanczos
from .mps import env_left, env_right, heff, ones_env, build_right_envs


def merge_mpo(W1, W2):
    """Two MPO sites as one: W[w, (s1 s2), (t1 t2), v] = sum_u W1[w, s1, t1, u] W2[u, s2, t2, v]."""
    wl, d1, _, _ = W1.shape
    _, d2, _, wr = W2.shape
    W = np.einsum("astu,ubcv->asbtcv", W1, W2)
    return W.reshape(wl, d1 * d2, d1 * d2, wr)


def svd_split(X, m):
    """Truncated SVD of the matrix X: (U[:, :m], S[:m], Vh[:m]), singular values descending."""
    U, S, Vh = np.linalg.svd(X, full_matrices=False)
    return U[:, :m], S[:m], Vh[:m], float(np.sum(S[m:] ** 2))


def ps2_step(mps, Ws, R, tau, kmax=20, tol=0.0, L=None, stats=None):
    n = len(mps)
    mps = [A.copy() for A in mps]
    R = list(R)
    L = [None] * (n + 1) if L is None else list(L)
    L[0] = ones_env()
    R[n] = ones_env()
    h = 0.5 * tau
    W2 = [merge_mpo(Ws[i], Ws[i + 1]) for i in range(n - 1)]
    discarded = []

    def two(i, X, z):
        return expm_lanczos(lambda x: heff(L[i], W2[i], R[i + 2], x), X, z, kmax=kmax, tol=tol)

    def one(i, C, z):
        return expm_lanczos(lambda x: heff(L[i], Ws[i], R[i + 1], x), C, z, kmax=kmax, tol=tol)

    def pair(i):
        ml, d1, m = mps[i].shape
        _, d2, mr = mps[i + 1].shape
        X = np.einsum("lsk,ktr->lstr", mps[i], mps[i + 1]).reshape(ml, d1 * d2, mr)
        return X, (ml, d1, m, d2, mr)

    # left-to-right half sweep
    for i in range(n - 1):
        last = i == n - 2
        X, (ml, d1, m, d2, mr) = pair(i)
        X = two(i, X, -1j * (tau if last else h))
        U, S, Vh, dw = svd_split(X.reshape(ml * d1, d2 * mr), m)
        discarded.append(dw)
        if last:
            mps[i] = (U * S).reshape(ml, d1, m)
            mps[i + 1] = Vh.reshape(m, d2, mr)
            R[i + 1] = env_right(R[i + 2], mps[i + 1], Ws[i + 1])
            break
        mps[i] = U.reshape(ml, d1, m)
        mps[i + 1] = (S[:, None] * Vh).reshape(m, d2, mr)
        L[i + 1] = env_left(L[i], mps[i], Ws[i])
        mps[i + 1] = one(i + 1, mps[i + 1], 1j * h)
    # right-to-left half sweep
    for i in range(n - 3, -1, -1):
        mps[i + 1] = one(i + 1, mps[i + 1], 1j * h)
        X, (ml, d1, m, d2, mr) = pair(i)
        X = two(i, X, -1j * h)
        U, S, Vh, dw = svd_split(X.reshape(ml * d1, d2 * mr), m)
        discarded.append(dw)
        mps[i] = (U * S).reshape(ml, d1, m)
        mps[i + 1] = Vh.reshape(m, d2, mr)
        R[i + 1] = env_right(R[i + 2], mps[i + 1], Ws[i + 1])
    if stats is not None:
        stats["discarded"] = discarded
    return mps, R, L


def evolve2(mps, Ws, tau, nsteps, kmax=20, tol=0.0, observe=None):
    """nsteps two-site PS steps from a right-canonical MPS (centre at site 0)."""
    R = build_right_envs(mps, Ws)
    out = []
    if observe is not None:
        out.append(observe(0.0, mps))
    for s in range(nsteps):
        mps, R, _ = ps2_step(mps, Ws, R, tau, kmax=kmax, tol=tol)
        if observe is not None:
            out.append(observe((s + 1) * tau, mps))
    return mps, out
