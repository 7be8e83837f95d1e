"""The largest chain at full size: 7 electronic sites x 30 modes x 10 levels
(217 sites), bond dimension 256.

* H[i] x and the left environment update at the shape of the widest
  vibrational site (M = 256, d = 10, the widest MPO channel dims of that
  chain), FP64 and FP32 contraction modes: sampled outputs against the
  oracle's single-element evaluation (the full application is too large for
  the oracle);
* one full TDVP-PS step of the chain in FP64: norm and energy conserved
  (properties of one-site TDVP-PS that hold at any size); FP32 contraction
  mode: populations within 1e-5 of the FP64 step.
"""

import numpy as np
import pytest

from inputs import draw_params, chain_sites, random_complex, workload
from inputs.randt import random_hermitian_env
from oracle import model, mps as om

from gpu_util import require_gpu, dev, host

pytestmark = pytest.mark.gpu

M = 256
NSAMPLE = 24


@pytest.fixture(scope="module")
def widest_site():
    p = draw_params(7, 30, 10, 0)
    sites = chain_sites(p)
    Ws, _ = model.mpo(p, sites)
    i = max((i for i, W in enumerate(Ws) if W.shape[1] == 10), key=lambda i: Ws[i].shape[0] * Ws[i].shape[3])
    return Ws[i]


@pytest.fixture(scope="module")
def ctxs():
    torch = require_gpu()
    from paper_1907_12044_amd import tdvp
    out = {}
    for name, prec in (("fp64", tdvp.FP64), ("fp32", tdvp.FP32)):
        c = tdvp.Context(0, prec)
        c.reserve(1 << 31)
        out[name] = c
    yield out
    torch.cuda.synchronize()


def _samples(shape, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(NSAMPLE)]


def _tol(prec):
    return 1e-12 if prec == "fp64" else 2e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_heff_at_full_size_sampled(ctxs, widest_site, prec):
    import torch
    from paper_1907_12044_amd import tdvp
    ctx = ctxs[prec]
    W = widest_site
    Wl, d, _, Wr = W.shape
    L = random_hermitian_env(M, Wl, 11)
    R = random_hermitian_env(M, Wr, 12)
    x = random_complex((M, d, M), 13)
    et = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "fp32":   # the oracle sees the same FP32-rounded environments
        L = L.astype(np.complex64).astype(np.complex128)
        R = R.astype(np.complex64).astype(np.complex128)
    y = dev(np.zeros_like(x))
    tdvp.heff_apply(ctx, dev(L, et), dev(W), dev(R, et), M, d, M, Wl, Wr, dev(x), y)
    yh = host(y)
    scale = np.abs(yh).max()
    for (b, s, q) in _samples((M, d, M), 14):
        ref = om.heff_element(L, W, R, x, b, s, q)
        assert abs(yh[b, s, q] - ref) < _tol(prec) * scale, (b, s, q)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_env_update_at_full_size_sampled(ctxs, widest_site, prec):
    import torch
    from paper_1907_12044_amd import tdvp
    ctx = ctxs[prec]
    W = widest_site
    Wl, d, _, Wr = W.shape
    L = random_hermitian_env(M, Wl, 21)
    A = random_complex((M, d, M), 22)
    et = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "fp32":
        L = L.astype(np.complex64).astype(np.complex128)
    out = dev(np.zeros((M, Wr, M)), et)
    tdvp.env_update(ctx, +1, dev(L, et), dev(A), dev(W), M, d, M, Wl, Wr, out)
    oh = host(out).astype(np.complex128)
    scale = np.abs(oh).max()
    for (q, y, r) in _samples((M, Wr, M), 23):
        ref = om.env_left_element(L, A, W, q, y, r)
        assert abs(oh[q, y, r] - ref) < _tol(prec) * scale, (q, y, r)


def test_full_step_conserves_norm_and_energy_fp32_populations():
    require_gpu()
    from paper_1907_12044_amd import tdvp
    p, sites, phys, dims, raw, w = workload("fmo7x30x10_M256")
    tau = w["dt_fs"] * model.AU_PER_FS
    run = tdvp.PsRun(p, sites, raw, 0, tdvp.FP64, kmax=20, graph=False)
    shift = run.mpo.shift
    e0 = run.observe_host().copy()
    run.step(tau, 1)
    o64 = run.observe_host().copy()
    del run
    # the centre keeps the norm exactly only as far as the 432 gauge shifts
    # of a step are orthonormal; the shifted Cholesky QR of these 2560 x 256
    # matrices is orthonormal to ~1e-12 each
    assert abs(e0[0] - 1.0) < 1e-11
    print(f"norm drift over one step: {abs(o64[0] - e0[0]):.2e}")
    assert abs(o64[0] - e0[0]) < 2e-9
    # energy of the shifted Hamiltonian (the large constant cancels)
    ea, eb = e0[1] - shift * e0[0], o64[1] - shift * o64[0]
    assert abs(eb - ea) < 1e-9 * max(abs(ea), 1.0)
    assert np.all(o64[2:] >= -1e-14)
    run32 = tdvp.PsRun(p, sites, raw, 0, tdvp.FP32, kmax=20, graph=False)
    run32.step(tau, 1)
    o32 = run32.observe_host()
    assert np.abs(o32[2:] - o64[2:]).max() < 1e-5
    assert abs(o32[0] - 1.0) < 1e-6
