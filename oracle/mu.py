"""TDVP-MU: TDVP with a fixed left-canonical gauge and matrix-unfolding
regularisation, integrated with the variable-mean-field scheme (Sec. II.A.2,
"TDVP-MU": eq:tdvp1_C, eq:tdvp1_L, eq:tdvp1_mu_rcano, eq:tdvp1_mu_L, eq:reg2).

State: left-canonical isometries L_0..L_{N-2} and the centre C_{N-1}.
Right-hand side at a given state:

1. left environments h[1:i] from the L's (eq:tdvp1_h1i);
2. an RQ sweep from the right end, C_{N-1} = D_{N-2} R_{N-1},
   L_{N-2} D_{N-2} = D_{N-3} R_{N-2}, ..., giving right-isometric R's (an
   orthonormal right basis) and the bond matrices D_i between sites i and
   i+1, so that the state at bond i reads |l_i[1:i]> D_i |r_i[i+1:N]>
   (the overlap of the left-continued basis is S[i+1:N] ~ D_i D_i^H);
   right environments in the orthonormal basis are built from the R's;
3. for every i < N-1, with D_i = U Lam V^H (SVD, eq:tdvp1_mu_rcano):
       G   = H[i] (L_i D_i)                      (H[i] with the R-basis environment)
       i dL_i/dt = (1 - L_i L_i^H) G V Lam~^{-1} U^H,
       Lam~ = Lam + sqrt(eps) exp(-Lam / sqrt(eps))       (eq:reg2)
   i.e. eq:tdvp1_mu_L after contracting its underlined factor to the identity;
4. i dC_{N-1}/dt = H[N-1] C_{N-1} (eq:tdvp1_C).

The coupled equations are integrated by the adaptive Dormand-Prince 5(4)
method (scipy.integrate.solve_ivp, "RK45"), as in the paper's VMF runs, or
by the second-order constant-mean-field scheme (mu_cmf_step, below).
Canonicality is not re-imposed during the integration.

Pins: at full bond dimension and full Schmidt rank the TDVP equations are
exact, so MU must follow exp(-iHt)psi (tests).  Agreement with TDVP-PS at
truncated bond dimension is stated by the paper only qualitatively: parity
unpinned, tolerance from measurement.  CMF: second-order convergence in tau
to the VMF solution at truncated bond dimension and to exp(-iHt)psi at full
bond dimension; norm and gauge kept to the integrator's tolerance (tests).
"""

from __future__ import annotations

import numpy as np
import scipy.integrate
import scipy.linalg

from .mps import qr_pos, env_left, env_right, heff, ones_env


def left_canonicalize(mps):
    """QR sweep 0 -> N-2 (eq:QR); centre left at site N-1, normalised."""
    m = [A.copy() for A in mps]
    for i in range(len(m) - 1):
        ml, d, mr = m[i].shape
        Q, R = qr_pos(m[i].reshape(ml * d, mr))
        m[i] = Q.reshape(ml, d, mr)
        m[i + 1] = np.einsum("kr,rtq->ktq", R, m[i + 1])
    m[-1] = m[-1] / np.linalg.norm(m[-1])
    return m


def mu_fields(mps, Ws, eps=1e-10):
    """The mean fields of every site at the state ``mps`` (steps 1-3 above).

    Entry i < N-1 is (Lenv_i, Renv_{i+1}, D_i, P_i) with P_i = V Lam~^{-1} U^H
    the regularised inverse factor of eq:tdvp1_mu_L; entry N-1 is
    (Lenv_{N-1}, ones, None, None).  Everything here depends on the state
    outside site i only through the environments and on the sites right of
    i through D_i: the quantities the constant-mean-field scheme holds fixed.
    """
    n = len(mps)
    L = [None] * (n + 1)
    L[0] = ones_env()
    for i in range(n - 1):
        L[i + 1] = env_left(L[i], mps[i], Ws[i])
    # RQ sweep: bond matrices D[i] between sites i, i+1 and right isometries
    D = [None] * n
    Rt = [None] * n
    Y = mps[n - 1]
    for i in range(n - 1, 0, -1):
        ml, d, mr = Y.shape
        Q, Rf = qr_pos(Y.reshape(ml, d * mr).conj().T)
        Rt[i] = Q.conj().T.reshape(ml, d, mr)
        D[i - 1] = Rf.conj().T                  # Y = D[i-1] R_i
        Y = np.einsum("lsk,kr->lsr", mps[i - 1], D[i - 1])
    Renv = [None] * (n + 1)
    Renv[n] = ones_env()
    for i in range(n - 1, 0, -1):
        Renv[i] = env_right(Renv[i + 1], Rt[i], Ws[i])
    se = np.sqrt(eps)
    fields = []
    for i in range(n - 1):
        U, lam, Vh = np.linalg.svd(D[i])
        lam_t = lam + se * np.exp(-lam / se)
        P = Vh.conj().T @ np.diag(1.0 / lam_t) @ U.conj().T
        fields.append((L[i], Renv[i + 1], D[i], P))
    fields.append((L[n - 1], Renv[n], None, None))
    return fields


def site_rhs(A, W, field):
    """d/dt of one site tensor with its mean field held fixed (step 3 or 4)."""
    Lenv, Renv, D, P = field
    if D is None:
        return -1j * heff(Lenv, W, Renv, A)
    ml, d, mr = A.shape
    C = np.einsum("lsk,kr->lsr", A, D)
    G = heff(Lenv, W, Renv, C).reshape(ml * d, mr)
    X = G @ P
    Am = A.reshape(ml * d, mr)
    X = X - Am @ (Am.conj().T @ X)
    return (-1j * X).reshape(ml, d, mr)


def mu_rhs(mps, Ws, eps=1e-10):
    """d/dt of every site tensor (list) for the left-canonical state ``mps``."""
    fields = mu_fields(mps, Ws, eps)
    return [site_rhs(A, W, f) for A, W, f in zip(mps, Ws, fields)]


def _pack(mps):
    return np.concatenate([A.reshape(-1) for A in mps])


def _unpack(y, shapes):
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(y[o:o + k].reshape(s))
        o += k
    return out


def mu_evolve(mps, Ws, t_final, eps=1e-10, rtol=1e-5, atol=1e-8, t_eval=None, max_step=np.inf):
    """Integrate the MU equations (VMF, RK45) from a left-canonical MPS.

    Returns (final MPS, list of MPS at t_eval if given, solver stats).
    """
    shapes = [A.shape for A in mps]

    def f(t, y):
        return _pack(mu_rhs(_unpack(y, shapes), Ws, eps))

    sol = scipy.integrate.solve_ivp(f, (0.0, t_final), _pack(mps).astype(np.complex128),
                                    method="RK45", rtol=rtol, atol=atol, t_eval=t_eval,
                                    max_step=max_step)
    if not sol.success:
        raise RuntimeError(sol.message)
    final = _unpack(sol.y[:, -1], shapes)
    snaps = [_unpack(sol.y[:, k], shapes) for k in range(sol.y.shape[1])] if t_eval is not None else []
    return final, snaps, {"nfev": sol.nfev}


# ---------------------------------------------------------------------------
# Constant mean field, second order (Sec. II.A.2, the CMF paragraph after
# eq:tdvp1_L_cano).  The mean fields of a site (its environments, and the
# bond matrix with its regularised inverse, i.e. H[i] and S[i+1:N]) are held
# fixed while the site tensor alone is integrated; each site's equation is
# then independent of the others.  Midpoint scheme: the fields of the state
# at t carry every site to t + tau/2; the fields of that midpoint state then
# carry every site of the state at t to t + tau.  The site tensors L_i obey
# a nonlinear equation (through the projector built from L_i itself) and are
# integrated by RK45; the centre obeys a linear one and is propagated by the
# exponential of its frozen effective Hamiltonian, which the paper computes
# by Krylov and this oracle computes exactly (a dense matrix exponential).

def _frozen_center(C, W, field, h):
    """exp(-i h H[N-1]) C with H[N-1] built from the frozen left environment."""
    Lenv, Renv, _, _ = field
    n = C.size
    Hm = np.empty((n, n), dtype=np.complex128)
    for k in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[k] = 1.0
        Hm[:, k] = heff(Lenv, W, Renv, e.reshape(C.shape)).reshape(-1)
    return (scipy.linalg.expm(-1j * h * Hm) @ C.reshape(-1)).reshape(C.shape)


def cmf_propagate(mps, Ws, fields, h, rtol=1e-10, atol=1e-12):
    """Every site carried over time h with the given frozen mean fields."""
    out = []
    n = len(mps)
    for i in range(n - 1):
        shape = mps[i].shape

        def f(t, y, W=Ws[i], fl=fields[i], shape=shape):
            return site_rhs(y.reshape(shape), W, fl).reshape(-1)

        sol = scipy.integrate.solve_ivp(f, (0.0, h), mps[i].reshape(-1).astype(np.complex128),
                                        method="RK45", rtol=rtol, atol=atol)
        if not sol.success:
            raise RuntimeError(sol.message)
        out.append(sol.y[:, -1].reshape(shape))
    out.append(_frozen_center(mps[n - 1], Ws[n - 1], fields[n - 1], h))
    return out


def mu_cmf_step(mps, Ws, tau, eps=1e-10, rtol=1e-10, atol=1e-12):
    """One second-order CMF step of length tau (midpoint mean fields)."""
    half = cmf_propagate(mps, Ws, mu_fields(mps, Ws, eps), 0.5 * tau, rtol, atol)
    return cmf_propagate(mps, Ws, mu_fields(half, Ws, eps), tau, rtol, atol)


def mu_cmf_evolve(mps, Ws, tau, nsteps, eps=1e-10, rtol=1e-10, atol=1e-12):
    m = [A.astype(np.complex128) for A in mps]
    for _ in range(nsteps):
        m = mu_cmf_step(m, Ws, tau, eps, rtol, atol)
    return m
