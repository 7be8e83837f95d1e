"""Two-site TDVP-PS on the GPU (tdvp_ps2_step) against the oracle
(oracle/ps2.py: ps2_step), through the C ABI.

* truncated bond dimension, 6- and 4-site chains: dense states after 3
  steps within 1e-10 of the oracle's, and the same discarded weight;
* full bond dimension: exact, against exp(-iHt) psi (the 4-site chain and
  the 6-site full-bond workload);
* the 21-site chain (7 electronic sites x 2 modes x 4 levels, M = 16):
  populations, norm and energy after 2 steps within 1e-10 of the oracle's
  (the norm carries the ~3e-6 weight that 80 truncated splits drop, summed
  in a different order on each side)
  (its dense state is too large to form; the SVD's singular vectors carry
  a free phase, so site tensors are compared through gauge-invariant
  observables);
* the split alone (tdvp_svd_split) against numpy's SVD on tall, square
  and wide matrices up to 64 x 64, both modes: truncated product,
  isometry and dropped weight;
* the merged MPO pair in the one-site H x and Lanczos kernels (d = 8);
* the limits: the one-work-group SVD refuses pairs wider than 64.
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw, workload
from oracle import model, mps as om, ps2, dense

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _run(p, sites, raw):
    from paper_1907_12044_amd import tdvp
    return tdvp.PsRun(p, sites, raw, 0, two_site=True, graph=False)


@pytest.mark.parametrize("n_e,n_modes,levels,M", [(3, 1, 4, 4), (3, 1, 4, 2), (2, 1, 3, 3)])
def test_ps2_matches_oracle_truncated(n_e, n_modes, levels, M):
    require_gpu()
    p = draw_params(n_e, n_modes, levels, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    raw = initial_mps_raw(p, M, 1e-1, 1)
    tau = 2 * model.AU_PER_FS
    run = _run(p, sites, raw)
    run.step(tau, 3)
    got = run.mps_numpy()
    dw_gpu = float(run.discarded.cpu().numpy()[0])
    m = om.right_canonicalize(raw)
    R = om.build_right_envs(m, Ws)
    dw = 0.0
    for _ in range(3):
        st = {}
        m, R, _ = ps2.ps2_step(m, Ws, R, tau, stats=st)
        dw += sum(st["discarded"])
    err = np.abs(om.mps_to_dense(got) - om.mps_to_dense(m)).max()
    print(f"two-site ({n_e},{n_modes},{levels}) M={M}: state difference {err:.2e}, "
          f"discarded {dw_gpu:.6e} vs {dw:.6e}")
    assert err < 1e-10
    assert abs(dw_gpu - dw) < 1e-12 + 1e-8 * dw


def test_ps2_full_bond_is_exact():
    require_gpu()
    p = draw_params(2, 1, 3, seed=4)
    sites = chain_sites(p)
    H, _ = model.dense_hamiltonian(p, sites)
    raw = initial_mps_raw(p, 6, 0.3, 2)
    T = 20 * model.AU_PER_FS
    run = _run(p, sites, raw)
    psi0 = om.mps_to_dense(run.mps_numpy())
    run.step(T / 10, 10)
    ref = dense.exact_evolve(H, psi0, [T])[0]
    err = np.abs(om.mps_to_dense(run.mps_numpy()) - ref).max()
    print(f"two-site full bond: {err:.2e} vs exp(-iHt) psi")
    assert err < 1e-10
    assert float(run.discarded.cpu().numpy()[0]) < 1e-20


def test_ps2_full_bond_workload_is_exact():
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo3x1x4_M16")
    H, _ = model.dense_hamiltonian(p, sites)
    run = _run(p, sites, raw)
    psi0 = om.mps_to_dense(run.mps_numpy())
    tau = w["dt_fs"] * model.AU_PER_FS
    run.step(tau, 10)
    ref = dense.exact_evolve(H, psi0, [10 * tau])[0]
    err = np.abs(om.mps_to_dense(run.mps_numpy()) - ref).max()
    print(f"two-site fmo3x1x4_M16, 10 steps: {err:.2e} vs exp(-iHt) psi")
    assert err < 1e-10


def test_ps2_21_sites_matches_oracle_observables():
    require_gpu()
    p, sites, phys, dims, raw, w = workload("fmo7x2x4_M16")
    Ws, _ = model.mpo(p, sites)
    tau = w["dt_fs"] * model.AU_PER_FS
    run = _run(p, sites, raw)
    run.step(tau, 2)
    got = run.mps_numpy()
    m = om.right_canonicalize(raw)
    R = om.build_right_envs(m, Ws)
    for _ in range(2):
        m, R, _ = ps2.ps2_step(m, Ws, R, tau)
    pg, po = om.site_populations(got, sites, p.n_e), om.site_populations(m, sites, p.n_e)
    ng, no = om.norm2(got), om.norm2(m)
    eg, eo = om.expectation_mpo(got, Ws).real, om.expectation_mpo(m, Ws).real
    print(f"two-site 21 sites: populations {np.abs(pg - po).max():.2e}, norm {abs(ng - no):.2e}, "
          f"energy {abs(eg - eo):.2e} (|E| {abs(eo):.2e})")
    assert np.abs(pg - po).max() < 1e-10
    assert abs(ng - no) < 1e-10      # both lose the same ~3e-6 to 80 truncations
    assert abs(eg - eo) < 1e-10 * max(abs(eo), 1e-3)


def test_ps2_rejects_pairs_beyond_the_svd():
    torch = require_gpu()
    from paper_1907_12044_amd import tdvp
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    Ws, wbond, shift = tdvp.fmo_model(p, sites)
    ctx = tdvp.Context(0, tdvp.FP64)
    mps = tdvp.DeviceMps(raw, ctx.device)
    mpo = tdvp.DeviceMpo(Ws, wbond, shift, ctx.device)
    with pytest.raises(tdvp.TdvpError, match="status 6"):     # 8 x 32 columns > 64
        tdvp.ps2_workspace_bytes(ctx, mps, mpo, 20)
    c32 = tdvp.Context(0, tdvp.FP32)
    with pytest.raises(tdvp.TdvpError, match="status 6"):     # FP64 only
        tdvp.ps2_workspace_bytes(c32, mps, mpo, 20)
    torch.cuda.synchronize()


@pytest.mark.parametrize("m,n,keep", [(2, 16, 2), (8, 8, 4), (8, 16, 4), (16, 8, 4), (8, 4, 4), (5, 7, 3),
                                      (64, 64, 32), (64, 16, 16)])
@pytest.mark.parametrize("mode", [0, 1])
def test_svd_split_matches_numpy(m, n, keep, mode):
    """tdvp_svd_split against numpy's SVD: the truncated product, the
    isometry of the kept vectors and the dropped weight (the singular
    vectors themselves carry a free phase)."""
    torch = require_gpu()
    from paper_1907_12044_amd import tdvp
    from inputs import random_complex
    from gpu_util import dev, host
    ctx = tdvp.Context(0, tdvp.FP64)
    X = random_complex((m, n), m * 100 + n)
    A = dev(np.zeros((m, keep), complex))
    B = dev(np.zeros((keep, n), complex))
    dw = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    tdvp.svd_split(ctx, dev(X), m, n, keep, mode, A, B, dw)
    torch.cuda.synchronize()
    a, b = host(A), host(B)
    U, S, Vh = np.linalg.svd(X, full_matrices=False)
    ref = (U[:, :keep] * S[:keep]) @ Vh[:keep]
    iso = a if mode == 0 else b.conj().T
    err = np.abs(a @ b - ref).max() / S[0]
    gram = np.abs(iso.conj().T @ iso - np.eye(keep)).max()
    print(f"svd_split {m}x{n} keep {keep} mode {mode}: product {err:.2e}, isometry {gram:.2e}")
    assert err < 1e-13
    assert gram < 1e-13
    assert abs(float(dw.cpu()[0]) - float(np.sum(S[keep:] ** 2))) < 1e-12 * float(np.sum(S ** 2))


def test_two_site_operator_matches_oracle():
    """The merged MPO pair of the 6-site chain in the one-site kernels:
    H x and the Lanczos propagator against the oracle's heff with
    merge_mpo, physical dimension d_i d_{i+1} = 8."""
    torch = require_gpu()
    from paper_1907_12044_amd import tdvp
    from inputs import random_complex
    from inputs.randt import random_hermitian_env
    from oracle.krylov import expm_lanczos
    from gpu_util import dev, host, relerr
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    ctx = tdvp.Context(0, tdvp.FP64)
    ctx.reserve(1 << 28)
    for i, (Ml, Mr) in enumerate([(1, 4), (2, 4), (4, 4)]):
        W2 = ps2.merge_mpo(Ws[i], Ws[i + 1])
        Wl, D, _, Wr = W2.shape
        L = random_hermitian_env(Ml, Wl, 10 + i)
        R = random_hermitian_env(Mr, Wr, 20 + i)
        x = random_complex((Ml, D, Mr), 30 + i)
        y = dev(np.zeros_like(x))
        tdvp.heff_apply(ctx, dev(L), dev(W2), dev(R), Ml, D, Mr, Wl, Wr, dev(x), y)
        e1 = relerr(host(y), om.heff(L, W2, R, x))
        xd = dev(x)
        kd = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        tdvp.lanczos_expm(ctx, dev(L), dev(W2), dev(R), Ml, D, Mr, Wl, Wr, -0.7j, 20, 0.0, xd, xd, kd)
        ref = expm_lanczos(lambda v: om.heff(L, W2, R, v), x, -0.7j, kmax=20)
        e2 = relerr(host(xd), ref)
        print(f"pair {i}: H x {e1:.2e}, Lanczos {e2:.2e}")
        assert e1 < 1e-12
        assert e2 < 1e-11
