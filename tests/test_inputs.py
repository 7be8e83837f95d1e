"""Checks on the seeded synthetic inputs (no method arithmetic lives there)."""

import numpy as np

from inputs import draw_params, chain_sites, bond_dims, initial_mps_raw, workload, WORKLOADS
from inputs.fmo import electronic_order, ensemble_bond
from oracle import mps as om


def _golden(name):
    import os
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, *vals = line.split()
                out[key] = [int(v) for v in vals]
    return out


def test_chain_matches_the_printed_fmo_chain():
    """Chain order and degree-of-freedom count printed for the paper's
    7-site model with 35 modes per site (tests/golden/fmo_chain.txt)."""
    g = _golden("fmo_chain.txt")
    assert [m + 1 for m in electronic_order(7)] == g["chain_order"]
    p = draw_params(7, g["modes_per_site"][0], 2, seed=0)
    sites = chain_sites(p)
    assert len(sites) == g["total_dofs"][0]
    assert sum(1 for s in sites if s[0] == "vib") == g["vibrational_dofs"][0]
    el = [s[1] + 1 for s in sites if s[0] == "el"]
    assert el == g["chain_order"]
    # every electronic site is followed by its own modes
    for i, s in enumerate(sites):
        if s[0] == "vib":
            owner = next(t for t in reversed(sites[:i]) if t[0] == "el")
            assert s[1] == owner[1]


def test_chain_order_matches_paper_for_seven_sites():
    # electronic sites in the order 7,5,3,1,2,4,6 (1-based), modes after their site
    assert [m + 1 for m in electronic_order(7)] == [7, 5, 3, 1, 2, 4, 6]
    p = draw_params(7, 2, 3, seed=0)
    sites = chain_sites(p)
    assert [s[0] for s in sites[:3]] == ["el", "vib", "vib"]
    assert sites[0][1] == 6 and sites[1][1] == 6


def test_draws_are_seeded_and_in_range():
    a = draw_params(7, 10, 8, seed=0)
    b = draw_params(7, 10, 8, seed=0)
    assert np.array_equal(a.E, b.E) and np.array_equal(a.J, b.J)
    assert np.all((a.E >= 12200) & (a.E <= 12600))
    iu = np.triu_indices(7, 1)
    assert np.all((np.abs(a.J[iu]) >= 5) & (np.abs(a.J[iu]) <= 100))
    assert np.array_equal(a.J, a.J.T) and np.all(np.diag(a.J) == 0)
    assert np.all((a.omega >= 100) & (a.omega <= 1600))
    assert np.all((a.S >= 0.01) & (a.S <= 0.1))
    r = draw_params(7, 10, 8, seed=0, realisation=3)
    assert np.array_equal(r.J, a.J) and not np.array_equal(r.E, a.E)
    assert ensemble_bond(0, 3) in (32, 64, 96, 128)


def test_bond_dims():
    assert bond_dims([2, 4, 2, 4, 2, 4], 16) == [1, 2, 8, 16, 8, 4, 1]


def test_initial_state_full_rank_and_one_exciton():
    p = draw_params(3, 1, 4, seed=0)
    sites = chain_sites(p)
    raw = initial_mps_raw(p, 8, 1e-2, 1)
    m = om.right_canonicalize(raw)
    psi = om.mps_to_dense(raw).reshape([s[3] for s in sites])
    psi = psi / np.linalg.norm(psi)
    # weight outside the one-exciton sector is zero
    occ = np.zeros(psi.shape, dtype=int)
    for pos, s in enumerate(sites):
        if s[0] == "el":
            shp = [1] * len(sites)
            shp[pos] = 2
            occ = occ + np.arange(2).reshape(shp)
    assert np.abs(psi[occ != 1]).max() == 0.0
    # every bond has full Schmidt rank well above round-off
    for b in range(1, len(sites)):
        s = np.linalg.svd(psi.reshape(int(np.prod(psi.shape[:b])), -1), compute_uv=False)
        assert s[m[b].shape[0] - 1] > 1e-9


def test_named_workloads_build():
    for name in ("fmo3x1x4_M16", "fmo7x10x8_M32"):
        p, sites, phys, dims, raw, w = workload(name)
        assert len(raw) == len(sites) == len(phys)
        for i, A in enumerate(raw):
            assert A.shape == (dims[i], phys[i], dims[i + 1])
    assert set(WORKLOADS) >= {"fmo3x1x4_M16", "fmo7x10x8_M32", "fmo7x10x8_M128"}
