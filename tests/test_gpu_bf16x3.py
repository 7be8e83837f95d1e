"""Split-BF16 contraction mode (TDVP_BF16X3): the tiled GEMMs of H[i]x, the
bond operator and the environment updates run on the bf16 matrix cores
with every FP32 operand split into two bf16 parts (FP32 accumulation).

* H[i]x and the bond operator vs the oracle on shapes spanning several 32-
  and 64-wide tiles with ragged tails: 1e-4 of the largest output (operands
  carry ~17 significant bits: 2^-16 per product, partly averaged over K);
* 77-site chain, M = 32, general path (fused step off, so every contraction
  goes through the split-BF16 GEMMs): populations within 1e-5 of the FP64
  oracle after three steps, norm conserved to 1e-6;
* same chain at M = 96 (general path by default): populations within 1e-5
  of the FP64 GPU path after two steps.
"""

import numpy as np
import pytest

from inputs import random_complex, random_mpo_like, workload
from inputs.randt import random_hermitian_env
from oracle import model, mps as om, ps

from gpu_util import require_gpu, dev, host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = require_gpu()
    from paper_1907_12044_amd import tdvp
    c = tdvp.Context(0, tdvp.BF16X3)
    c.reserve(1 << 30)
    yield c
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [(7, 2, 13, 3, 4), (40, 8, 33, 9, 5), (96, 10, 100, 5, 3), (128, 8, 128, 9, 9)])
def test_heff_apply_bf16x3(ctx, shape):
    import torch
    from paper_1907_12044_amd import tdvp
    Ml, d, Mr, Wl, Wr = shape
    seed = sum(shape) + 100
    L = random_hermitian_env(Ml, Wl, seed).astype(np.complex64).astype(np.complex128)
    R = random_hermitian_env(Mr, Wr, seed + 1).astype(np.complex64).astype(np.complex128)
    W = random_mpo_like(Wl, d, Wr, seed + 2, density=0.4)
    x = random_complex((Ml, d, Mr), seed + 3)
    y = dev(np.zeros_like(x))
    tdvp.heff_apply(ctx, dev(L, torch.complex64), dev(W), dev(R, torch.complex64), Ml, d, Mr, Wl, Wr,
                    dev(x), y)
    assert relerr(host(y), om.heff(L, W, R, x)) < 1e-4


@pytest.mark.parametrize("Ml,Mr,W", [(16, 16, 5), (33, 40, 9), (128, 128, 9)])
def test_bond_operator_bf16x3(ctx, Ml, Mr, W):
    import torch
    from paper_1907_12044_amd import tdvp
    L = random_hermitian_env(Ml, W, Ml + 50).astype(np.complex64).astype(np.complex128)
    R = random_hermitian_env(Mr, W, Mr + 51).astype(np.complex64).astype(np.complex128)
    D = random_complex((Ml, Mr), Ml + Mr + 52)
    y = dev(np.zeros_like(D))
    tdvp.heff_apply(ctx, dev(L, torch.complex64), None, dev(R, torch.complex64), Ml, 1, Mr, W, W, dev(D), y)
    assert relerr(host(y), om.bond_op(L, R, D)) < 1e-4


def test_fmo77_m32_general_path_populations_within_1e5():
    require_gpu()
    from paper_1907_12044_amd import tdvp
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M32")
    tau = w["dt_fs"] * model.AU_PER_FS
    run = tdvp.PsRun(p, sites, raw, 0, tdvp.BF16X3, kmax=20, fused=False)
    run.step(tau, 3)
    obs = run.observe_host()
    Ws, _ = model.mpo(p, sites)
    m, _ = ps.evolve(om.right_canonicalize(raw), Ws, tau, 3, kmax=20)
    pops = om.site_populations(m, sites, p.n_e)
    err = np.abs(obs[2:] - pops).max()
    print(f"split-BF16 vs FP64 oracle, max population difference after 3 steps: {err:.2e}")
    assert err < 1e-5
    assert abs(obs[0] - 1.0) < 1e-6


def test_fmo77_m96_populations_within_1e5_of_fp64():
    require_gpu()
    from paper_1907_12044_amd import tdvp
    p, sites, phys, dims, raw, w = workload("fmo7x10x8_M96")
    tau = w["dt_fs"] * model.AU_PER_FS
    out = {}
    for prec in (tdvp.FP64, tdvp.BF16X3):
        run = tdvp.PsRun(p, sites, raw, 0, prec, kmax=20)
        run.step(tau, 2)
        out[prec] = run.observe_host().copy()
        del run
    err = np.abs(out[tdvp.BF16X3][2:] - out[tdvp.FP64][2:]).max()
    print(f"split-BF16 vs FP64 GPU, M = 96, max population difference after 2 steps: {err:.2e}")
    assert err < 1e-5
