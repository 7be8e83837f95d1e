"""Pins for the oracle's TDVP-PS step (eq:ps_trotter, eq:tdvp2_C, eq:tdvp2_D).

* full bond dimension: the split step is exact, so it must equal exp(-iHt)psi
  (every backward factor cancels a forward one with the same projector, and
  the factor that is left has projector 1);
* truncated bond dimension: equal to the same splitting applied literally to
  the dense state with dense projectors (no environments, no Krylov space);
* norm and energy are conserved exactly (each factor is unitary with a
  Hermitian generator P H P and the state stays in the range of P);
* time reversibility: the step with -tau undoes the step with tau;
* second order: the one-step error against a fine-step run falls as tau^3;
* g = 0 electronic-only chain: populations |[exp(-i H1 t)]_{m,1}|^2 with
  H1 = diag(E) + J (textbook single-exciton dynamics).
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw, workload
from oracle import model, mps as om, ps, dense


def _setup(n_e, n_modes, levels, M, eta, seed=0, phi_seed=1, coupling=True):
    p = draw_params(n_e, n_modes, levels, seed=seed, coupling=coupling)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    mps = om.right_canonicalize(initial_mps_raw(p, M, eta, phi_seed))
    return p, sites, Ws, mps


def test_full_bond_dimension_is_exact():
    p, sites, phys, dims, raw, w = workload("fmo3x1x4_M16")
    Ws, _ = model.mpo(p, sites)
    H, _ = model.dense_hamiltonian(p, sites)
    mps = om.right_canonicalize(raw)
    psi0 = om.mps_to_dense(mps)
    tau = w["dt_fs"] * model.AU_PER_FS
    m, _ = ps.evolve(mps, Ws, tau, w["steps"], kmax=20)
    ref = dense.exact_evolve(H, psi0, [w["steps"] * tau])[0]
    assert np.abs(om.mps_to_dense(m) - ref).max() < 1e-10


@pytest.mark.parametrize("n_e,n_modes,levels,M", [(2, 1, 3, 2), (2, 1, 3, 3), (3, 1, 2, 3)])
def test_truncated_equals_dense_projector_splitting(n_e, n_modes, levels, M):
    p, sites, Ws, mps = _setup(n_e, n_modes, levels, M, 0.3)
    H, _ = model.dense_hamiltonian(p, sites)
    dims = [s[3] for s in sites]
    tau = 3.0 * model.AU_PER_FS
    psi, pL, pR = dense.dense_projector_init(mps)
    R = om.build_right_envs(mps, Ws)
    m = mps
    for _ in range(3):
        m, R, _ = ps.ps_step(m, Ws, R, tau)
        psi, pL, pR = dense.dense_projector_ps_step(psi, pL, pR, H, dims, tau)
    assert np.abs(om.mps_to_dense(m) - psi).max() < 1e-12
    # and the truncation is real: the result differs from exact propagation
    ex = dense.exact_evolve(H, om.mps_to_dense(mps), [3 * tau])[0]
    assert np.abs(psi - ex).max() > 1e-6


def test_truncated_c1_shape_one_step_dense_projector():
    p, sites, Ws, mps = _setup(3, 1, 4, 4, 1e-2)
    H, _ = model.dense_hamiltonian(p, sites)
    dims = [s[3] for s in sites]
    tau = model.AU_PER_FS
    psi, pL, pR = dense.dense_projector_init(mps)
    R = om.build_right_envs(mps, Ws)
    m, R, _ = ps.ps_step(mps, Ws, R, tau)
    psi, pL, pR = dense.dense_projector_ps_step(psi, pL, pR, H, dims, tau)
    assert np.abs(om.mps_to_dense(m) - psi).max() < 1e-12


@pytest.mark.parametrize("M", [2, 4, 8])
def test_norm_and_energy_conserved(M):
    p, sites, Ws, mps = _setup(3, 1, 4, M, 1e-2)
    e0 = om.expectation_mpo(mps, Ws).real
    tau = model.AU_PER_FS
    m, _ = ps.evolve(mps, Ws, tau, 20, kmax=20)
    assert om.norm2(m) == pytest.approx(1.0, abs=1e-12)
    assert om.expectation_mpo(m, Ws).real == pytest.approx(e0, abs=1e-12 * max(abs(e0), 1e-3))


def test_time_reversible():
    p, sites, Ws, mps = _setup(3, 1, 4, 4, 1e-1)
    tau = 2.0 * model.AU_PER_FS
    R = om.build_right_envs(mps, Ws)
    m1, R1, _ = ps.ps_step(mps, Ws, R, tau)
    m2, _, _ = ps.ps_step(m1, Ws, R1, -tau)
    assert np.abs(om.mps_to_dense(m2) - om.mps_to_dense(mps)).max() < 1e-10


def test_second_order_in_tau():
    p, sites, Ws, mps = _setup(3, 1, 4, 4, 1e-1)
    T = 8.0 * model.AU_PER_FS

    def run(nsteps):
        m, _ = ps.evolve(mps, Ws, T / nsteps, nsteps, kmax=20)
        return om.mps_to_dense(m)

    ref = run(64)
    errs = [np.linalg.norm(run(n) - ref) for n in (2, 4, 8)]
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < s < 2.3 for s in slopes), (errs, slopes)


def test_g0_electronic_chain_matches_single_exciton_closed_form():
    n_e = 7
    p = draw_params(n_e, 0, 2, seed=0, coupling=False)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    mps = om.right_canonicalize(initial_mps_raw(p, 8, 0.0))     # full M for 7 two-level sites
    E = p.E * model.HARTREE_PER_CM
    H1 = np.diag(E - E.mean()) + p.J * model.HARTREE_PER_CM
    lam, V = np.linalg.eigh(H1)
    tau = 2.0 * model.AU_PER_FS
    nsteps = 10
    m, _ = ps.evolve(mps, Ws, tau, nsteps, kmax=20)
    t = nsteps * tau
    U = V @ np.diag(np.exp(-1j * lam * t)) @ V.conj().T
    ref = np.abs(U[:, 0]) ** 2
    pops = om.site_populations(m, sites, n_e)
    assert np.abs(pops - ref).max() < 1e-10
