"""The autotuner (tdvp_set_autotune): candidate launch shapes compute the same
quantities, so a tuned run agrees with an untuned one to round-off; the
step that meets new problem keys runs eagerly, later steps replay a graph
built with the chosen shapes.

* 77-site chain, M = 32, FP64 (fused Lanczos step; the environment-update
  and centre-move GEMMs tuned): three steps, populations / norm / energy
  within 1e-10 of the untuned run and of the oracle's first step;
* same chain at M = 96, FP32 contractions (GEMM tiles tuned on the general
  path): populations within 1e-6 of the untuned run after two steps.
"""

import numpy as np
import pytest

from inputs import workload
from oracle import model, mps as om, ps

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _runs(name, precision):
    from paper_1907_12044_amd import tdvp
    p, sites, phys, dims, raw, w = workload(name)
    tuned = tdvp.PsRun(p, sites, raw, 0, precision, kmax=20, autotune=True)
    plain = tdvp.PsRun(p, sites, raw, 0, precision, kmax=20, autotune=False)
    return p, sites, raw, w, tuned, plain


def test_autotuned_fused_path_matches_untuned_and_oracle():
    require_gpu()
    from paper_1907_12044_amd import tdvp
    p, sites, raw, w, tuned, plain = _runs("fmo7x10x8_M32", tdvp.FP64)
    tau = w["dt_fs"] * model.AU_PER_FS
    tuned.step(tau, 1)
    assert tdvp.autotune_count(tuned.ctx) > 0
    assert tdvp.autotune_count(plain.ctx) == 0
    first = tuned.observe_host().copy()
    tuned.step(tau, 2)                     # graph replay with the tuned shapes
    plain.step(tau, 3)
    a, b = tuned.observe_host(), plain.observe_host()
    assert np.abs(a - b).max() < 1e-10 * max(1.0, np.abs(b).max())
    # the first tuned step against the oracle's step
    Ws, _ = model.mpo(p, sites)
    m, _ = ps.evolve(om.right_canonicalize(raw), Ws, tau, 1, kmax=20)
    pops = om.site_populations(m, sites, p.n_e)
    assert np.abs(first[2:] - pops).max() < 1e-10


def test_autotuned_general_path_fp32_matches_untuned():
    require_gpu()
    from paper_1907_12044_amd import tdvp
    p, sites, raw, w, tuned, plain = _runs("fmo7x10x8_M96", tdvp.FP32)
    tau = w["dt_fs"] * model.AU_PER_FS
    tuned.step(tau, 2)
    plain.step(tau, 2)
    assert tdvp.autotune_count(tuned.ctx) > 0
    a, b = tuned.observe_host(), plain.observe_host()
    assert np.abs(a[2:] - b[2:]).max() < 1e-6
    assert abs(a[0] - 1.0) < 1e-6
