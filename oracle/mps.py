"""MPS primitives in plain numpy (Sec. II.A).

Layouts: an MPS site tensor is (M_left, d, M_right); an MPO site tensor is
(W_left, d_out, d_in, W_right); an environment is (M, W, M) indexed
[bra, mpo channel, ket] with the bra conjugated (eq:tdvp1_h).
Bonds are numbered 0..N: site i sits between bonds i and i+1.  L[b] is the
contraction of sites 0..b-1 (h[1:b] in the paper's 1-based notation), R[b]
that of sites b..N-1 (h[b+1:N]); L[0] = R[N] = 1.
"""

from __future__ import annotations

import numpy as np


def qr_pos(A):
    """Thin QR A = Q R with diag(R) real and >= 0 (eq:QR)."""
    Q, R = np.linalg.qr(A, mode="reduced")
    dg = np.diag(R)
    ph = np.ones_like(dg)
    nz = np.abs(dg) > 0
    ph[nz] = dg[nz] / np.abs(dg[nz])
    return Q * ph[None, :], R * np.conj(ph)[:, None]


def qr_cholesky3(A):
    """Thin QR A = Q R (m >= n) by shifted Cholesky QR in three passes
    (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci.
    Comput. 42 (2020)): W_0 = A; pass p: G = W_p^H W_p, R_p = chol(G [+ s I])
    with G = R_p^H R_p, W_{p+1} = W_p R_p^{-1}; the first pass adds the shift
    s = 11 (m n + n (n + 1)) u tr(G), u = 2^-53.  Q = W_3, R = R_3 R_2 R_1
    (upper triangular, real positive diagonal: the factorisation of eq:QR,
    unique for full-rank A).  A second backward-stable QR for the oracle:
    on numerically rank-deficient site tensors two such QRs choose
    different (equally valid) bases for the negligible directions, and the
    one-site TDVP-PS trajectory can amplify that difference."""
    m, n = A.shape
    W = A
    Rt = np.eye(n, dtype=complex)
    for p in range(3):
        G = W.conj().T @ W
        if p == 0:
            G = G + 11.0 * (m * n + n * (n + 1)) * 2.0 ** -53 * np.trace(G).real * np.eye(n)
        Rp = np.linalg.cholesky(G).conj().T           # G = Rp^H Rp
        W = np.linalg.solve(Rp.T, W.T).T              # W Rp^{-1}
        Rt = Rp @ Rt
    return W, Rt


def right_canonicalize(mps, qr=qr_pos):
    """RQ sweep N-1 -> 1 (eq:QR, mirrored); then normalise the centre at site 0."""
    mps = [A.copy() for A in mps]
    for i in range(len(mps) - 1, 0, -1):
        ml, d, mr = mps[i].shape
        C = mps[i].reshape(ml, d * mr)
        Q, Rf = qr(C.conj().T)              # C^H = Q Rf  ->  C = Rf^H Q^H
        mps[i] = Q.conj().T.reshape(ml, d, mr)
        mps[i - 1] = np.einsum("lsk,kr->lsr", mps[i - 1], Rf.conj().T)
    mps[0] = mps[0] / np.linalg.norm(mps[0])
    return mps


# Each contraction below is the single einsum given in its docstring, carried
# out as a chain of pairwise tensordot calls (small tensors contracted one by
# one, as Sec. II.A.2 prescribes); the chain is only an evaluation order.

def env_left(L, A, W):
    """h[1:i] from h[1:i-1] (eq:tdvp1_h1i with eq:tdvp1_h, A = L^{sigma}).

    einsum("bwk,ktr,wsty,bsq->qyr", L, A, W, conj(A))
    """
    T = np.tensordot(L, A, axes=([2], [0]))                 # b w t r
    T = np.tensordot(T, W, axes=([1, 2], [0, 2]))           # b r s y
    T = np.tensordot(A.conj(), T, axes=([0, 1], [0, 2]))    # q r y
    return np.ascontiguousarray(np.transpose(T, (0, 2, 1)))


def env_right(R, A, W):
    """h[i:N] from h[i+1:N] (eq:tdvp1_hiN with eq:tdvp1_h, A = R^{sigma}).

    einsum("qyr,ktr,wsty,bsq->bwk", R, A, W, conj(A))
    """
    T = np.tensordot(A, R, axes=([2], [2]))                 # k t q y
    T = np.tensordot(T, W, axes=([1, 3], [2, 3]))           # k q w s
    T = np.tensordot(A.conj(), T, axes=([1, 2], [3, 1]))    # b k w
    return np.ascontiguousarray(np.transpose(T, (0, 2, 1)))


def heff(L, W, R, x):
    """H[i] x with H[i] = h[1:i-1] W[i] h[i+1:N] (eq:tdvp1_H, eq:tdvp2_C).

    einsum("bwk,wstv,qvr,ktr->bsq", L, W, R, x)
    """
    T = np.tensordot(x, R, axes=([2], [2]))                 # k t q v
    T = np.tensordot(W, T, axes=([2, 3], [1, 3]))           # w s k q
    return np.tensordot(L, T, axes=([1, 2], [0, 2]))        # b s q


def heff_element(L, W, R, x, b, s, q):
    """One element (b, s, q) of H[i] x (eq:tdvp1_H): the sum over w, k, t, v,
    r of L[b, w, k] W[w, s, t, v] R[q, v, r] x[k, t, r], evaluated on its own
    so that single outputs of a large application can be checked.
    """
    T = np.tensordot(x, R[q], axes=([2], [1]))              # k t v
    T = np.tensordot(W[:, s], T, axes=([1, 2], [1, 2]))     # w k
    return complex(np.sum(L[b] * T))


def env_left_element(L, A, W, q, y, r):
    """One element (q, y, r) of the left environment update (eq:tdvp1_h1i):
    the sum over b, w, k, t, s of L[b, w, k] A[k, t, r] W[w, s, t, y] conj(A[b, s, q]).
    """
    T = np.tensordot(L, A[:, :, r], axes=([2], [0]))        # b w t
    T = np.tensordot(T, W[:, :, :, y], axes=([1, 2], [0, 2]))   # b s
    return complex(np.sum(np.conj(A[:, :, q]) * T))


def env_right_element(R, A, W, b, w, k):
    """One element (b, w, k) of the right environment update (eq:tdvp1_hiN):
    the sum over q, y, r, t, s of R[q, y, r] A[k, t, r] W[w, s, t, y] conj(A[b, s, q]).
    """
    T = np.tensordot(A[k], R, axes=([1], [2]))              # t q y
    T = np.tensordot(W[w], T, axes=([1, 2], [0, 2]))        # s q
    return complex(np.sum(np.conj(A[b]) * T))


def bond_op(L, R, D):
    """Zero-site operator of eq:tdvp2_D: sum_w h[1:i]_{l' w l} h[i+1:N]_{r' w r} D_{l r}.

    einsum("bwk,qwr,kr->bq", L, R, D)
    """
    T = np.tensordot(D, R, axes=([1], [2]))                 # k q w
    return np.tensordot(L, T, axes=([1, 2], [2, 0]))        # b q


def ones_env():
    return np.ones((1, 1, 1), dtype=np.complex128)


def build_right_envs(mps, Ws):
    """R[b] for b = N..1 from right-canonical sites (R[0] left as None)."""
    n = len(mps)
    R = [None] * (n + 1)
    R[n] = ones_env()
    for i in range(n - 1, 0, -1):
        R[i] = env_right(R[i + 1], mps[i], Ws[i])
    return R


def build_left_envs(mps, Ws):
    n = len(mps)
    L = [None] * (n + 1)
    L[0] = ones_env()
    for i in range(n):
        L[i + 1] = env_left(L[i], mps[i], Ws[i])
    return L


def _transfer(E, A, B):
    """einsum("bk,ksr,bsq->qr", E, A, conj(B)): one step of <B|A> from the left."""
    T = np.tensordot(E, A, axes=([1], [0]))                 # b s r
    return np.tensordot(B.conj(), T, axes=([0, 1], [0, 1]))  # q r


def norm2(mps):
    """<psi|psi> by a full transfer pass (no gauge assumed)."""
    E = np.ones((1, 1), dtype=np.complex128)
    for A in mps:
        E = _transfer(E, A, A)
    return float(E[0, 0].real)


def expectation_mpo(mps, Ws):
    """<psi|O|psi> for an MPO O by a full transfer pass (no gauge assumed)."""
    L = ones_env()
    for A, W in zip(mps, Ws):
        L = env_left(L, A, W)
    return complex(L[0, 0, 0])


def site_populations(mps, sites, n_e):
    """P_m = <psi| a+_m a_m |psi> for every electronic site m (not divided by the norm).

    One full transfer pass per site with the number operator inserted, so the
    result does not depend on the gauge of the MPS.
    """
    pops = np.zeros(n_e)
    for p, s in enumerate(sites):
        if s[0] != "el":
            continue
        E = np.ones((1, 1), dtype=np.complex128)
        for i, A in enumerate(mps):
            if i == p:
                B = A.copy()
                B[:, 0, :] = 0.0                   # n = |1><1|
                E = _transfer(E, B, A)
            else:
                E = _transfer(E, A, A)
        pops[s[1]] = float(E[0, 0].real)
    return pops


def mps_to_dense(mps):
    """Contract an MPS into its full state vector (site 0 slowest)."""
    psi = mps[0].reshape(-1, mps[0].shape[2])
    for A in mps[1:]:
        psi = np.einsum("pk,ksr->psr", psi, A).reshape(-1, A.shape[2])
    return psi.reshape(-1)
