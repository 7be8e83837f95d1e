"""Parity of the full TDVP-PS step on the GPU (tdvp_ps_step) with the oracle.

* 3 electronic sites x 1 mode x 4 levels, full bond dimension 16, 50 steps of
  1 fs: equal to exact propagation exp(-iHt) psi(0) (and to the oracle);
* the same chain at truncated bond dims 4 and 8: equal to the oracle's
  dense state after 20 steps;
* 7 x 10 x 8 (77 sites), M = 32, 2 fs: populations, norm and energy equal to
  the oracle's after 3 steps (1e-10), and, at the full run length the
  benchmark uses, norm and energy conserved (properties that hold at any size);
* FP32 contraction mode on the same chain: populations within 1e-5 of the
  FP64 oracle.
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw, workload
from oracle import model, mps as om, ps, dense

from gpu_util import require_gpu, host

pytestmark = pytest.mark.gpu


def _gpu_run(p, sites, raw, precision=0, kmax=20, tol=0.0, graph=True, fused=True):
    from paper_1907_12044_amd import tdvp
    return tdvp.PsRun(p, sites, raw, 0, precision, kmax, tol, graph=graph, fused=fused)


def _oracle_init(p, sites, raw):
    Ws, _ = model.mpo(p, sites)
    return Ws, om.right_canonicalize(raw)


def test_canonical_form_matches_oracle():
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    run = _gpu_run(p, sites, raw)
    g = run.mps_numpy()
    _, o = _oracle_init(p, sites, raw)
    # full-rank bonds: the right-canonical form with real positive R diagonals is unique
    err = max(np.abs(a - b).max() for a, b in zip(g, o))
    assert err < 1e-8
    assert om.norm2(g) == pytest.approx(1.0, abs=1e-13)


def test_full_bond_dimension_equals_exact_propagation():
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo3x1x4_M16")
    H, _ = model.dense_hamiltonian(p, sites)
    tau = w["dt_fs"] * model.AU_PER_FS
    run = _gpu_run(p, sites, raw)
    psi0 = om.mps_to_dense(run.mps_numpy())
    run.step(tau, w["steps"])
    psi = om.mps_to_dense(run.mps_numpy())
    ref = dense.exact_evolve(H, psi0, [w["steps"] * tau])[0]
    assert np.abs(psi - ref).max() < 1e-10
    obs = run.observe_host()
    pops_ref = om.site_populations(run.mps_numpy(), sites, p.n_e)
    assert np.abs(obs[2:] - pops_ref).max() < 1e-12
    assert obs[0] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("M", [4, 8])
def test_truncated_bond_dimension_equals_oracle(M):
    require_gpu()
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    raw = initial_mps_raw(p, M, 1e-2, 1)
    tau = model.AU_PER_FS
    run = _gpu_run(p, sites, raw)
    run.step(tau, 20)
    Ws, m0 = _oracle_init(p, sites, raw)
    m, _ = ps.evolve(m0, Ws, tau, 20, kmax=20)
    assert np.abs(om.mps_to_dense(run.mps_numpy()) - om.mps_to_dense(m)).max() < 1e-10


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "general"])
def test_fmo77_m32_fp64_matches_oracle(fused):
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    tau = w["dt_fs"] * model.AU_PER_FS
    nsteps = 3
    run = _gpu_run(p, sites, raw, fused=fused)
    e0 = run.observe_host().copy()
    run.step(tau, nsteps)
    obs = run.observe_host()
    Ws, m0 = _oracle_init(p, sites, raw)
    m, _ = ps.evolve(m0, Ws, tau, nsteps, kmax=20)
    pops = om.site_populations(m, sites, p.n_e)
    E = om.expectation_mpo(m, Ws).real
    shift = model.shifted_terms(p, sites)[4]
    assert np.abs(obs[2:] - pops).max() < 1e-10
    assert abs(obs[0] - om.norm2(m)) < 1e-12
    assert abs((obs[1] - shift * obs[0]) - E) < 1e-10 * max(abs(E), model.HARTREE_PER_CM)
    # gauge-invariant overlap of the two states
    g = run.mps_numpy()
    ov = np.ones((1, 1), complex)             # ov[a, b]: a the GPU bond, b the oracle bond
    for A, B in zip(g, m):
        ov = np.tensordot(np.tensordot(ov, A, axes=([0], [0])), B.conj(), axes=([0, 1], [0, 1]))
    assert 1.0 - abs(ov[0, 0]) < 1e-10
    # the step conserves norm and energy
    assert abs(obs[0] - e0[0]) < 1e-12 and abs(obs[1] - e0[1]) < 1e-9 * abs(e0[1])


def test_fmo77_m32_full_length_conserves_norm_and_energy():
    """The run length of this workload (500 steps of 2 fs = 1 ps), in the
    launch configuration the benchmark times (graph replay)."""
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    tau = w["dt_fs"] * model.AU_PER_FS
    run = _gpu_run(p, sites, raw)
    e0 = run.observe_host().copy()
    run.step(tau, w["steps"])
    obs = run.observe_host()
    assert abs(obs[0] - 1.0) < 1e-11
    # shifted energy (the large constant cancels) conserved to round-off
    shift = run.mpo.shift
    assert abs((obs[1] - shift * obs[0]) - (e0[1] - shift * e0[0])) < 1e-11
    assert np.all(obs[2:] >= -1e-14)


def test_fmo77_m32_fp32_populations_within_1e5():
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    tau = w["dt_fs"] * model.AU_PER_FS
    nsteps = 3
    run = _gpu_run(p, sites, raw, precision=1)
    run.step(tau, nsteps)
    obs = run.observe_host()
    Ws, m0 = _oracle_init(p, sites, raw)
    m, _ = ps.evolve(m0, Ws, tau, nsteps, kmax=20)
    pops = om.site_populations(m, sites, p.n_e)
    assert np.abs(obs[2:] - pops).max() < 1e-5
    assert abs(obs[0] - 1.0) < 1e-6


def test_graph_replays_equal_eager_steps():
    """Every replay of the captured step equals the eager step, bit for bit."""
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    tau = w["dt_fs"] * model.AU_PER_FS
    eager = _gpu_run(p, sites, raw, graph=False)
    graph = _gpu_run(p, sites, raw, graph=True)
    for s in range(4):
        eager.step(tau, 1)
        a = eager.observe_host()
        graph.step(tau, 1)
        b = graph.observe_host()
        assert np.array_equal(a, b), (s, a, b)
        ma, mb = eager.mps_numpy(), graph.mps_numpy()
        assert all(np.array_equal(x, y) for x, y in zip(ma, mb)), s


def test_parity_drift_over_steps():
    """FP64 GPU vs oracle populations at 1, 3 and 5 steps (10 fs, inside the
    horizon where two FP64 runs agree to round-off; records the drift)."""
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    tau = w["dt_fs"] * model.AU_PER_FS
    run = _gpu_run(p, sites, raw)
    Ws, m = _oracle_init(p, sites, raw)
    R = om.build_right_envs(m, Ws)
    done = 0
    for target in (1, 3, 5):
        run.step(tau, target - done)
        for _ in range(target - done):
            m, R, _ = ps.ps_step(m, Ws, R, tau)
        done = target
        obs = run.observe_host()
        err = np.abs(obs[2:] - om.site_populations(m, sites, p.n_e)).max()
        print(f"steps {target}: max population difference {err:.3e}")
        assert err < 1e-10


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_fmo77_m64_one_step_matches_oracle(precision):
    """Bond dim 64 (multi-work-group QR path; in FP32 the fused Lanczos
    step): one step against the oracle, 1e-10 (FP64) or 1e-5 (FP32)."""
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M64")
    tau = w["dt_fs"] * model.AU_PER_FS
    run = _gpu_run(p, sites, raw, precision=precision)
    run.step(tau, 1)
    obs = run.observe_host()
    Ws, m0 = _oracle_init(p, sites, raw)
    m, _ = ps.evolve(m0, Ws, tau, 1, kmax=20)
    pops = om.site_populations(m, sites, p.n_e)
    if precision == 0:
        assert np.abs(obs[2:] - pops).max() < 1e-10
        assert abs(obs[0] - om.norm2(m)) < 1e-12
    else:
        assert np.abs(obs[2:] - pops).max() < 1e-5
        assert abs(obs[0] - om.norm2(m)) < 1e-6


def test_fmo77_m128_mixed_vs_fp64_gpu():
    """Bond dim 128: FP32 contractions against the FP64 GPU path over the
    first 3 steps, plus norm and energy conservation (the oracle comparison
    of this chain is in test_gpu_goldens.py)."""
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M128")
    tau = w["dt_fs"] * model.AU_PER_FS
    r64 = _gpu_run(p, sites, raw, precision=0)
    r32 = _gpu_run(p, sites, raw, precision=1)
    e0 = r64.observe_host().copy()
    for s in range(3):
        r64.step(tau, 1)
        r32.step(tau, 1)
        a, b = r64.observe_host(), r32.observe_host()
        print(f"step {s + 1}: |dP| {np.abs(a[2:] - b[2:]).max():.2e}  |dnorm| {abs(a[0] - b[0]):.2e}")
        assert np.abs(a[2:] - b[2:]).max() < 1e-5
    assert abs(a[0] - 1.0) < 1e-11
    shift = r64.mpo.shift
    assert abs((a[1] - shift * a[0]) - (e0[1] - shift * e0[0])) < 1e-10
