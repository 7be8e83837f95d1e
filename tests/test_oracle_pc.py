"""Pins for the oracle's P&C-RK4 (oracle/pc.py: eq:RK4, eq:mpo-apply,
eq:mps+mps, eq:QR, eq:SVD).

* MPO x MPS equals H psi, MPS + MPS equals the sum (dense, brute force);
* compression is exact when each bond keeps the state's Schmidt rank (a
  sum of two product states compressed to bond dimension 2), and at full
  bond dimension on a general state;
* full bond dimension: one step equals sum_{k<=4} (-i H tau)^k / k! psi
  (RK4 on a linear, time-independent equation), and the error against
  exp(-i H t) psi falls at fourth order in tau.
"""

import numpy as np

from inputs import draw_params, chain_sites, initial_mps_raw
from oracle import model, mps as om, pc, dense


def _case(M=6, eta=0.3):
    p = draw_params(2, 1, 3, seed=4)
    sites = chain_sites(p)
    H, _ = model.dense_hamiltonian(p, sites)
    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(initial_mps_raw(p, M, eta, 2))
    return p, sites, H, Ws, m


def test_mpo_apply_and_mps_add_match_dense():
    _, _, H, Ws, m = _case()
    psi = om.mps_to_dense(m)
    assert np.abs(om.mps_to_dense(pc.mpo_apply(Ws, m)) - H @ psi).max() < 1e-14 * max(np.abs(H).max(), 1.0) * 10
    m2 = [A * (0.3 + 0.1j) for A in m]
    got = om.mps_to_dense(pc.mps_add(m, m2))
    assert np.abs(got - (psi + om.mps_to_dense(m2))).max() < 1e-14


def test_compression_exact_at_the_schmidt_rank():
    _, _, H, Ws, m = _case()
    bonds = [1] + [A.shape[2] for A in m]
    psi = om.mps_to_dense(m)
    full = pc.compress(pc.mps_add(m, m), bonds)
    assert np.abs(om.mps_to_dense(full) - 2 * psi).max() < 1e-13
    # two product states: Schmidt rank 2 at every bond
    rng = np.random.default_rng(3)
    dims = [A.shape[1] for A in m]
    a = [rng.standard_normal((1, d, 1)) + 1j * rng.standard_normal((1, d, 1)) for d in dims]
    b = [rng.standard_normal((1, d, 1)) + 1j * rng.standard_normal((1, d, 1)) for d in dims]
    s = pc.mps_add(a, b)
    c = pc.compress(s, [1] + [2] * (len(dims) - 1) + [1])
    assert max(A.shape[2] for A in c[:-1]) <= 2
    assert np.abs(om.mps_to_dense(c) - om.mps_to_dense(s)).max() < 1e-13


def test_full_bond_step_is_the_fourth_order_taylor_polynomial():
    _, _, H, Ws, m = _case()
    bonds = [1] + [A.shape[2] for A in m]
    psi = om.mps_to_dense(m)
    tau = 2.0 * model.AU_PER_FS
    got = om.mps_to_dense(pc.pc_rk4_step(m, Ws, tau, bonds))
    ref = np.zeros_like(psi)
    term = psi.copy()
    for k in range(5):
        ref = ref + term
        term = (-1j * tau / (k + 1)) * (H @ term)
    assert np.abs(got - ref).max() < 1e-12


def test_full_bond_converges_at_fourth_order():
    _, _, H, Ws, m = _case()
    bonds = [1] + [A.shape[2] for A in m]
    T = 20 * model.AU_PER_FS
    ref = dense.exact_evolve(H, om.mps_to_dense(m), [T])[0]
    errs = []
    for nst in (10, 20, 40):
        errs.append(np.abs(om.mps_to_dense(pc.pc_rk4_evolve(m, Ws, T / nst, nst, bonds)) - ref).max())
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0, errs
