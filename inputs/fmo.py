"""Synthetic FMO-like exciton-vibration chains (Frenkel-Holstein model).

The paper's model (Sec. II.C, eq:holstein) is a 7-site FMO complex whose site
energies, couplings and discretised spectral density come from the
literature.  Those numbers are not available here, so every parameter is
drawn from fixed distributions with a seeded PCG64 generator, in a fixed
draw order:

1. site energies  E[n_e]              ~ U(12200, 12600) cm^-1
2. |J| for i<j in row-major order     ~ U(5, 100) cm^-1
3. the sign of each J (same order)    equiprobable +-1
4. mode frequencies omega[n_e, nm]    ~ U(100, 1600) cm^-1
5. Huang-Rhys factors S[n_e, nm]      ~ U(0.01, 0.1)   (g = sqrt(S))

Chain ordering (Sec. II.C): electronic sites in the order odd-descending
then even-ascending (for 7 sites: 7,5,3,1,2,4,6), each followed directly by
its own vibrational modes.  Electronic sites have local dimension 2
(|0> empty, |1> one exciton); a mode truncated to ``levels`` has the number
basis |0>..|levels-1>.

Nothing here evolves a state; :func:`initial_mps_raw` only places numbers
into tensors.  Canonicalisation and normalisation are left to the consumer.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class ChainParams:
    n_e: int
    n_modes: int
    levels: int
    E: np.ndarray          # (n_e,) cm^-1
    J: np.ndarray          # (n_e, n_e) cm^-1, symmetric, zero diagonal
    omega: np.ndarray      # (n_e, n_modes) cm^-1
    S: np.ndarray          # (n_e, n_modes) Huang-Rhys factors
    seed: int = 0
    realisation: Optional[int] = None
    extra: dict = field(default_factory=dict)


def draw_params(n_e: int, n_modes: int, levels: int, seed: int = 0,
                realisation: Optional[int] = None,
                disorder_sigma: float = 100.0,
                coupling: bool = True) -> ChainParams:
    """Draw model parameters in the fixed order stated in the module doc.

    ``realisation`` r >= 0 adds static disorder E_m += N(0, sigma) drawn from
    ``default_rng([seed, r])``.  ``coupling=False`` zeroes the Huang-Rhys
    factors after drawing them (the g = 0 limit), keeping the other draws
    identical.
    """
    rng = np.random.default_rng(seed)
    E = rng.uniform(12200.0, 12600.0, size=n_e)
    npair = n_e * (n_e - 1) // 2
    mag = rng.uniform(5.0, 100.0, size=npair)
    sign = np.where(rng.integers(0, 2, size=npair) == 0, -1.0, 1.0)
    J = np.zeros((n_e, n_e))
    k = 0
    for i in range(n_e):
        for j in range(i + 1, n_e):
            J[i, j] = J[j, i] = sign[k] * mag[k]
            k += 1
    omega = rng.uniform(100.0, 1600.0, size=(n_e, n_modes))
    S = rng.uniform(0.01, 0.1, size=(n_e, n_modes))
    if not coupling:
        S = np.zeros_like(S)
    if realisation is not None:
        rr = np.random.default_rng([seed, realisation])
        E = E + rr.normal(0.0, disorder_sigma, size=n_e)
    return ChainParams(n_e, n_modes, levels, E, J, omega, S, seed, realisation)


def electronic_order(n_e: int) -> List[int]:
    """0-based electronic site indices in chain order (odd desc, even asc, 1-based)."""
    odd = [m for m in range(n_e, 0, -1) if m % 2 == 1]
    even = [m for m in range(1, n_e + 1) if m % 2 == 0]
    return [m - 1 for m in odd + even]


def chain_sites(p: ChainParams):
    """List of chain sites as tuples ('el', m, None, 2) or ('vib', m, lam, levels)."""
    sites = []
    for m in electronic_order(p.n_e):
        sites.append(("el", m, None, 2))
        for lam in range(p.n_modes):
            sites.append(("vib", m, lam, p.levels))
    return sites


def bond_dims(phys: List[int], M: int) -> List[int]:
    """Bond dims M_b = min(M, prod(d[:b]), prod(d[b:])), M_0 = M_N = 1."""
    n = len(phys)
    out = [1]
    for b in range(1, n):
        left = 1
        for d in phys[:b]:
            left = min(left * d, M)
        right = 1
        for d in phys[b:]:
            right = min(right * d, M)
        out.append(min(M, left, right))
    out.append(1)
    return out


def _sector_counts(sites, b):
    """(#el sites, product of vib dims) on each side of bond b, dims capped."""
    cap = 1 << 40
    nel_l = sum(1 for s in sites[:b] if s[0] == "el")
    nel_r = sum(1 for s in sites[b:] if s[0] == "el")
    vl = 1
    for s in sites[:b]:
        if s[0] == "vib":
            vl = min(vl * s[3], cap)
    vr = 1
    for s in sites[b:]:
        if s[0] == "vib":
            vr = min(vr * s[3], cap)
    # left states with q excitons (q in {0,1}); right states with 1-q excitons
    left = {0: vl, 1: nel_l * vl}
    right = {0: vr, 1: nel_r * vr}
    return left, right


# Highest vibrational level of a mode that the random block of the initial
# state touches.
VIB_BLOCK_LEVEL = 2


def initial_mps_raw(p: ChainParams, M: int, eta: float = 0.0,
                    phi_seed: int = 1, exciton_site: int = 0):
    """Raw initial MPS tensors (M_b, d, M_{b+1}) complex128, not canonical.

    eta == 0: the Hartree product state (exciton on electronic site
    ``exciton_site``, every mode in |0>), zero-padded to the bond dims.

    eta > 0: the product state plus two small parts that fill every bond
    index, so that the bond bases are fixed by the state rather than by how
    a QR completes a rank-deficient matrix:
      * bond index 0 carries the product state;
      * bond index 1 (where the one-exciton sector allows it) carries the
        zero-phonon exciton on the other electronic sites: the state
        eta * sum_{m != exciton_site} a_m |exciton on m, every mode in |0>>,
        a_m seeded complex normal, is a bond-dimension-2 MPS whose two
        channels are bond indices 0 and 1 (index 1 holds the channel whose
        exciton number differs from the product state's);
      * the other indices hold a seeded random block:
          A[0, s, k]  = eta * G_in   (leave the product channel)
          A[j, s, k]  = G_blk        (random block, O(1) entries)
          A[j, s, 0]  = G_out        (return to the product channel)
          A[1, s, k]  = G_w          (leave the zero-phonon channel)
        so every path through the block carries weight ~eta: it leaves the
        product channel with weight eta, or the zero-phonon channel (weight
        1 where that channel itself has weight eta, eta where it has 1).
    The zero-phonon channel holds the states that carry the exciton from
    site to site (without it the one-site integrator has no basis state to
    move population into); the random block gives the vibrational
    excitations room.  No channel is reached only through two small
    couplings, so the smallest Schmidt values scale with eta, not eta^2,
    and the populations at t = 0 stay within ~1e-6 of the product state's
    (pinned per workload in tests/test_inputs.py).  All random entries are
    graded by exciton number: every bond index carries a label q in {0,1}
    (excitons to its left) and an entry is nonzero only when the labels
    match the local exciton number, so the state lies in the one-exciton
    sector.
    """
    sites = chain_sites(p)
    phys = [s[3] for s in sites]
    n = len(sites)
    dims = bond_dims(phys, M)

    def occ(s):  # product-state local level
        return 1 if (s[0] == "el" and s[1] == exciton_site) else 0

    prod = []
    for i, s in enumerate(sites):
        A = np.zeros((dims[i], phys[i], dims[i + 1]), dtype=np.complex128)
        A[0, occ(s), 0] = 1.0
        prod.append(A)
    if eta == 0.0:
        return prod

    # exciton-number labels of every bond index; has_w[b]: bond index 1 is
    # the zero-phonon channel (label 1 - product label)
    prod_q = [0] * (n + 1)
    q = 0
    for i, s in enumerate(sites):
        q += occ(s)
        prod_q[i + 1] = q
    labels = [[0]]
    has_w = [False] * (n + 1)
    for b in range(1, n):
        m = dims[b]
        left, right = _sector_counts(sites, b)
        cap = {qq: min(left[qq], right[1 - qq]) for qq in (0, 1)}
        n0 = min(cap[0], m // 2)
        n1 = min(cap[1], m - n0)
        if n0 + n1 < m:
            n0 = min(cap[0], m - n1)
        pq = prod_q[b]
        cnt = {0: n0, 1: n1}
        if n0 + n1 < m or cnt[pq] < 1:
            raise ValueError(f"bond {b}: one-exciton sector too small for M={M}")
        cnt[pq] -= 1
        lab = [pq]
        if m >= 2 and cnt[1 - pq] >= 1:
            has_w[b] = True
            cnt[1 - pq] -= 1
            lab.append(1 - pq)
        lab += [0] * cnt[0] + [1] * cnt[1]
        labels.append(lab)
    labels.append([1])

    # The random block keeps modes at levels <= VIB_BLOCK_LEVEL (low phonon
    # numbers, as the small Huang-Rhys factors favour), except on modes next
    # to a bond whose capped space on either side is too small to fill it
    # (near the chain ends), which use every level.
    def capped_dim(sl):
        nel = sum(1 for t in sl if t[0] == "el")
        v = 1
        for t in sl:
            if t[0] == "vib":
                v = min(v * min(t[3], VIB_BLOCK_LEVEL + 1), 1 << 40)
        return (1 + nel) * v
    fits = [True] + [capped_dim(sites[:b]) >= 2 * dims[b] and capped_dim(sites[b:]) >= 2 * dims[b]
                     for b in range(1, n)] + [True]
    capped = [fits[i] and fits[i + 1] for i in range(n)]

    rng = np.random.default_rng(phi_seed)
    a = (rng.standard_normal(p.n_e) + 1j * rng.standard_normal(p.n_e)) / np.sqrt(2.0)
    out = []
    for i, s in enumerate(sites):
        d = phys[i]
        lq = np.asarray(labels[i])
        rq = np.asarray(labels[i + 1])
        shape = (len(lq), d, len(rq))
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        G = (re + 1j * im) / np.sqrt(2.0)
        nloc = np.arange(d) if s[0] == "el" else np.zeros(d, dtype=int)
        mask = lq[:, None, None] + nloc[None, :, None] == rq[None, None, :]
        if s[0] == "vib" and capped[i]:
            mask &= (np.arange(d) <= VIB_BLOCK_LEVEL)[None, :, None]
        # expected squared norm of every row (j, :, :) is 1
        w2 = mask.sum(axis=(1, 2))
        G = np.where(mask, G, 0.0) / np.sqrt(np.maximum(w2, 1))[:, None, None]
        jl = 2 if has_w[i] else 1        # first random-block index, left bond
        jr = 2 if has_w[i + 1] else 1    # first random-block index, right bond
        A = prod[i].copy()
        A[0, :, jr:] = eta * G[0, :, jr:]
        if jl == 2:
            # leave the zero-phonon channel: left of the exciton site it is
            # the placed exciton (weight eta), right of it the exciton not
            # placed yet (weight 1, so its paths must pay eta here)
            A[1, :, jr:] = (1.0 if prod_q[i] == 0 else eta) * G[1, :, jr:]
        A[jl:, :, jr:] = G[jl:, :, jr:]
        A[jl:, :, 0] = G[jl:, :, 0]
        # zero-phonon channel: E = exciton not placed yet, F = placed
        wl, wr = has_w[i], has_w[i + 1]
        if s[0] == "vib":
            if wl and wr:
                A[1, 0, 1] = 1.0
        elif occ(s):                       # E -> F through the product channel
            if wl:
                A[1, 0, 0] = 1.0           # F (placed on the left) passes
            if wr:
                A[0, 0, 1] = 1.0           # E passes, placed on the right
        elif prod_q[i] == 0:               # left of the exciton site: 0 = E, 1 = F
            if wr:
                A[0, 1, 1] = eta * a[s[1]]
            if wl and wr:
                A[1, 0, 1] = 1.0
        else:                              # right of it: 0 = F, 1 = E
            if wl:
                A[1, 1, 0] = eta * a[s[1]]
            if wl and wr:
                A[1, 0, 1] = 1.0
        out.append(A)
    return out


# Named workloads, by the model and run sizes they stand for.
WORKLOADS = {
    # 3 electronic sites x 1 mode x 4 levels, full bond dimension, exact product state
    "fmo3x1x4_M16": dict(n_e=3, n_modes=1, levels=4, M=16, dt_fs=1.0, steps=50,
                         seed=0, eta=0.0),
    # 7 electronic sites x 10 modes x 8 levels, M = 32, FP64
    "fmo7x10x8_M32": dict(n_e=7, n_modes=10, levels=8, M=32, dt_fs=2.0, steps=500,
                          seed=0, eta=1e-4, phi_seed=1),
    # the same chain at the other bond dimensions of the disorder ensemble
    "fmo7x10x8_M64": dict(n_e=7, n_modes=10, levels=8, M=64, dt_fs=2.0, steps=500,
                          seed=0, eta=1e-4, phi_seed=1),
    "fmo7x10x8_M96": dict(n_e=7, n_modes=10, levels=8, M=96, dt_fs=2.0, steps=500,
                          seed=0, eta=1e-4, phi_seed=1),
    # same chain at M = 128, mixed precision, Krylov dim 20
    "fmo7x10x8_M128": dict(n_e=7, n_modes=10, levels=8, M=128, dt_fs=2.0, steps=1000,
                           seed=0, eta=1e-4, phi_seed=1, kdim=20),
    # 7 electronic sites x 2 modes x 4 levels, M = 16: small enough for the
    # two-site step's one-work-group SVD (bond x phys <= 64 at every pair)
    "fmo7x2x4_M16": dict(n_e=7, n_modes=2, levels=4, M=16, dt_fs=1.0, steps=50,
                         seed=0, eta=1e-2, phi_seed=1),
    # 7 electronic sites x 30 modes x 10 levels, M = 256
    # (217 sites: more points where the random part can leave the product
    # channel, so a smaller eta keeps the t = 0 populations within 1e-6)
    "fmo7x30x10_M256": dict(n_e=7, n_modes=30, levels=10, M=256, dt_fs=1.0, steps=200,
                            seed=0, eta=7e-5, phi_seed=1),
}


def ensemble_bond(seed: int, r: int) -> int:
    """Bond dimension of disorder realisation r, uniform over {32, 64, 96, 128}."""
    rr = np.random.default_rng([seed, r, 1])
    return int((32, 64, 96, 128)[rr.integers(0, 4)])


# The static-disorder ensemble: realisations of the 77-site chain with site
# energies perturbed by N(0, 100 cm^-1) and bond dimensions drawn from
# {32, 64, 96, 128}; the initial state of every member is built like the
# single-chain workloads' (same eta and random block seed).
ENSEMBLE = dict(n_e=7, n_modes=10, levels=8, dt_fs=2.0, steps=500, seed=0, eta=1e-4,
                phi_seed=1, kdim=20, nreal=64)


def ensemble_members(nreal: int = 64, seed: int = 0):
    """[(r, params, M_r, raw initial MPS)] for realisations r = 0..nreal-1."""
    e = ENSEMBLE
    out = []
    for r in range(nreal):
        p = draw_params(e["n_e"], e["n_modes"], e["levels"], seed, realisation=r)
        M = ensemble_bond(seed, r)
        out.append((r, p, M, initial_mps_raw(p, M, e["eta"], e["phi_seed"])))
    return out


def workload(name: str):
    """Return (params, sites, phys, bond dims, raw initial MPS, run settings)."""
    w = dict(WORKLOADS[name])
    p = draw_params(w["n_e"], w["n_modes"], w["levels"], w["seed"])
    sites = chain_sites(p)
    phys = [s[3] for s in sites]
    dims = bond_dims(phys, w["M"])
    mps = initial_mps_raw(p, w["M"], w.get("eta", 0.0), w.get("phi_seed", 1))
    return p, sites, phys, dims, mps, w
