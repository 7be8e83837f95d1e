"""Batched ensemble (tdvp_ps_step_batched): every kernel covers all
instances in one launch; each instance must come out exactly as the single
chain run does (same kernels, same tile shapes, same reduction order)."""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, initial_mps_raw
from oracle import model

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _instances(nb, M, n_modes=3, levels=4):
    ps_ = [draw_params(4, n_modes, levels, seed=0, realisation=r) for r in range(nb)]
    sites = chain_sites(ps_[0])
    raws = [initial_mps_raw(p, M, 1e-2, 10 + r) for r, p in enumerate(ps_)]
    return ps_, sites, raws


@pytest.mark.parametrize("precision,graph,M", [(0, True, 12), (0, False, 12), (1, True, 12), (0, True, 48)],
                         ids=["fp64-graph", "fp64-eager", "fp32-graph", "fp64-graph-M48"])
def test_batched_equals_single_runs(precision, graph, M):
    """M = 12: register QR and fused Lanczos step, split the same way for one
    or three chains, so batched == single bit for bit.  M = 48 (4 modes x 8
    levels): also the Cholesky QR path (384 x 48 gauge shifts).  There the
    fused step splits a column over fewer work-groups for three chains than
    for one, so a single run differs in summation order: its observables
    agree to 1e-12, and each instance is compared bit for bit with instance
    0 of an ensemble of three copies of the same realisation (same count,
    hence the same split), which shows that instances do not interact."""
    require_gpu()
    from paper_1907_12044_amd import tdvp
    nb = 3
    ps_, sites, raws = (_instances(nb, M) if M == 12 else _instances(nb, M, n_modes=4, levels=8))
    tau = 2.0 * model.AU_PER_FS
    ens = tdvp.PsEnsemble(ps_, sites, raws, 0, precision, kmax=20, graph=graph)
    singles = [tdvp.PsRun(p, sites, raw, 0, precision, kmax=20, graph=graph) for p, raw in zip(ps_, raws)]
    exact = M == 12
    copies = [] if exact else [tdvp.PsEnsemble([p] * nb, sites, [raw] * nb, 0, precision, kmax=20, graph=graph)
                               for p, raw in zip(ps_, raws)]
    for step in range(3):
        ens.step(tau, 1)
        ob = ens.observe_host()
        for r, run in enumerate(singles):
            run.step(tau, 1)
            o1 = run.observe_host()
            if exact:
                assert np.array_equal(ob[r], o1), (step, r, ob[r], o1)
            else:
                assert np.abs(ob[r] - o1).max() < 1e-12, (step, r, ob[r], o1)
                copies[r].step(tau, 1)
                oc = copies[r].observe_host()
                assert np.array_equal(ob[r], oc[0]), (step, r, ob[r], oc[0])
    for r in range(nb):
        a = ens.mps_numpy(r)
        b = singles[r].mps_numpy() if exact else copies[r].mps_numpy(0)
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), r


def test_batched_rejects_unstrided_layout():
    require_gpu()
    from paper_1907_12044_amd import tdvp
    import ctypes
    ps_, sites, raws = _instances(3, 8)
    ens = tdvp.PsEnsemble(ps_, sites, raws, 0, 0, kmax=8)
    mps_arr, mpo_arr, env_arr = ens.descs
    # swap two instances: still valid descriptors, but not at constant strides
    bad = (type(mps_arr))(mps_arr[0], mps_arr[2], mps_arr[1])
    with pytest.raises(tdvp.TdvpError):
        tdvp.ps_step_batched(ens.ctx, (bad, mpo_arr, env_arr), 1.0)
