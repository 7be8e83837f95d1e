"""Checks on the seeded synthetic inputs (no method arithmetic lives there)."""

import numpy as np
import pytest

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


@pytest.mark.parametrize("name", ["fmo7x10x8_M32", "fmo7x10x8_M64", "fmo7x10x8_M96", "fmo7x10x8_M128"])
def test_initial_populations_within_1e6_of_the_product_state(name):
    """The small parts that fill the bond channels move the t = 0
    populations of the normalised state by at most 1e-6 from the Hartree
    product state (exciton on electronic site 1), at every bond dimension;
    the state stays in the one-exciton sector (populations sum to 1)."""
    p, sites, phys, dims, raw, w = workload(name)
    m = om.right_canonicalize(raw)
    pops = om.site_populations(m, sites, p.n_e)
    dev = np.abs(pops - np.eye(p.n_e)[0]).max()
    assert dev < 1e-6, dev
    assert dev > 1e-9        # the channels really are filled
    assert abs(pops.sum() - 1.0) < 1e-12


def test_initial_state_of_the_217_site_chain_from_its_golden():
    """Same bound for the 217-site chain, read from the step-0 record of the
    oracle run stored in tests/golden/c5.npz (too large to redo here)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c5.npz")
    if not os.path.exists(path):
        pytest.skip("c5 golden not generated")
    g = np.load(path)
    assert int(g["steps"][0]) == 0
    dev = np.abs(g["pops"][0] - np.eye(7)[0]).max()
    assert 1e-9 < dev < 1e-6, dev
