"""Frenkel-Holstein Hamiltonian of the FMO-like chain (Sec. II.C, eq:holstein).

    H = sum_m E_m n_m + sum_{m != n} J_mn a+_m a_n
        + sum_{m,l} w_ml (b+ b + 1/2) + sum_{m,l} g_ml w_ml (b+ + b) n_m

Electronic sites are two-level (hard-core exciton, a+ = |1><0|, no string
operator: only the one-exciton sector is ever populated).  Modes use the
truncated number basis, b|k> = sqrt(k)|k-1>.  g = sqrt(S) with S the
Huang-Rhys factor.  Energies are converted from cm^-1 to hartree, time from
fs to atomic units.

Constant offsets are removed from the operator that is evolved: the zero
point sum_ml w_ml / 2 (a multiple of the identity) and Ebar * N_exc with Ebar
the mean site energy (a constant on the one-exciton sector).  They are
returned as ``shift`` so that E = <H'> + shift * <psi|psi>.

Two independent constructions are given: :func:`dense_hamiltonian` (explicit
Kronecker products, tiny chains only) and :func:`mpo` (a left-indexed
finite-state construction; one channel per open operator, bond dim
2 + 2k + [inside a vibrational block] with k the electronic sites to the left).
"""

from __future__ import annotations

import numpy as np

HARTREE_PER_CM = 4.556335252767e-6     # 1 cm^-1 in hartree
AU_PER_FS = 41.341373335               # 1 fs in atomic units of time


def local_ops(d):
    """Creation/annihilation/number for a d-level site (a for d=2, b otherwise)."""
    a = np.diag(np.sqrt(np.arange(1, d, dtype=float)), k=1).astype(np.complex128)
    ad = a.conj().T
    num = np.diag(np.arange(d, dtype=float)).astype(np.complex128)
    return ad, a, num


def shifted_terms(params, sites):
    """Per-term coefficients in hartree, and the removed constant."""
    E = params.E * HARTREE_PER_CM
    J = params.J * HARTREE_PER_CM
    w = params.omega * HARTREE_PER_CM
    g = np.sqrt(params.S)
    Ebar = float(np.mean(E))
    shift = Ebar + 0.5 * float(np.sum(w))
    return E - Ebar, J, w, g, shift


def dense_hamiltonian(params, sites):
    """Dense H' (shifted) on the full chain space, site 0 the slowest index."""
    eps, J, w, g, shift = shifted_terms(params, sites)
    dims = [s[3] for s in sites]
    D = int(np.prod(dims))

    def embed(ops):
        """Kronecker product with the given {position: operator}, identity elsewhere."""
        out = np.ones((1, 1), dtype=np.complex128)
        for i, d in enumerate(dims):
            out = np.kron(out, ops.get(i, np.eye(d)))
        return out

    pos_el = {s[1]: i for i, s in enumerate(sites) if s[0] == "el"}
    H = np.zeros((D, D), dtype=np.complex128)
    ad2, a2, n2 = local_ops(2)
    for m, p in pos_el.items():
        H += eps[m] * embed({p: n2})
    for m, p in pos_el.items():
        for n_, q in pos_el.items():
            if m != n_ and J[m, n_] != 0.0:
                H += J[m, n_] * embed({p: ad2, q: a2})
    for i, s in enumerate(sites):
        if s[0] != "vib":
            continue
        m, lam, d = s[1], s[2], s[3]
        bd, b, nb = local_ops(d)
        H += w[m, lam] * embed({i: nb})
        H += g[m, lam] * w[m, lam] * embed({i: bd + b, pos_el[m]: n2})
    return H, shift


def mpo(params, sites):
    """MPO tensors W[i] of shape (W_i, d_out, d_in, W_{i+1}) for H' (shifted).

    Channels on bond b: 'ready' (nothing placed yet), 'done' (a whole term
    placed), ('cre', m) / ('ann', m) for every electronic site m left of b
    that still has an electronic partner right of b, and ('num', m) while b
    lies inside the vibrational block that follows electronic site m.
    The first bond keeps only 'ready', the last only 'done'.
    """
    eps, J, w, g, shift = shifted_terms(params, sites)
    n = len(sites)
    el_pos = [i for i, s in enumerate(sites) if s[0] == "el"]

    def channels(b):
        if b == 0:
            return ["ready"]
        if b == n:
            return ["done"]
        ch = ["ready"]
        left_el = [sites[i][1] for i in el_pos if i < b]
        right_any = any(i >= b for i in el_pos)
        if right_any:
            for m in left_el:
                ch += [("cre", m), ("ann", m)]
        prev = sites[b - 1]
        nxt = sites[b]
        owner = prev[1]
        if nxt[0] == "vib" and nxt[1] == owner:
            ch.append(("num", owner))
        ch.append("done")
        return ch

    chans = [channels(b) for b in range(n + 1)]
    Ws = []
    for i, s in enumerate(sites):
        d = s[3]
        L, R = chans[i], chans[i + 1]
        W = np.zeros((len(L), d, d, len(R)), dtype=np.complex128)
        I = np.eye(d, dtype=np.complex128)
        ad, a, num = local_ops(d)

        def put(lc, rc, op):
            if lc in L and rc in R:
                W[L.index(lc), :, :, R.index(rc)] += op

        put("ready", "ready", I)
        put("done", "done", I)
        # channels that only pass through this site
        for c in L:
            if isinstance(c, tuple) and c in R and c[0] in ("cre", "ann"):
                put(c, c, I)
        if s[0] == "el":
            m = s[1]
            put("ready", "done", eps[m] * num)
            put("ready", ("cre", m), ad)
            put("ready", ("ann", m), a)
            for c in L:
                if isinstance(c, tuple) and c[0] == "cre":
                    put(c, "done", J[c[1], m] * a)      # J_km a+_k a_m
                if isinstance(c, tuple) and c[0] == "ann":
                    put(c, "done", J[m, c[1]] * ad)     # J_mk a+_m a_k
            put("ready", ("num", m), num)
        else:
            m, lam = s[1], s[2]
            put("ready", "done", w[m, lam] * num)
            put(("num", m), "done", g[m, lam] * w[m, lam] * (ad + a))
            put(("num", m), ("num", m), I)
        Ws.append(W)
    return Ws, shift


def mpo_to_dense(Ws):
    """Contract an MPO into its dense matrix (brute force, tiny chains)."""
    T = Ws[0][0]                       # (d, d, W1)
    T = np.transpose(T, (2, 0, 1))     # (W, dout, din)
    for W in Ws[1:]:
        # T[w, O, I] W[w, o, i, v] -> T'[v, (O o), (I i)]
        T = np.einsum("wOI,woiv->vOoIi", T, W)
        v, O, o, I_, i = T.shape
        T = T.reshape(v, O * o, I_ * i)
    return T[0]
