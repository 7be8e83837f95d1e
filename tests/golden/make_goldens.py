"""Write the stored expected values of the full-size GPU parity tests.

Every value written here comes from the CPU oracle (``oracle/``) on the
seeded synthetic inputs of ``inputs/``; nothing else is imported.  Each
target writes one ``tests/golden/<target>.npz`` (plain arrays, no pickled
objects) holding the observables or sampled outputs the GPU tests compare
with, plus a ``meta`` string that records how it was made.

Targets (run one per process, e.g. ``python tests/golden/make_goldens.py c2``):

  c2        77-site chain, M = 32, dt = 2 fs: norm, shifted energy and
            populations after every step up to step 500 (the full run)
  c3        the same chain at M = 128: the first 50 steps
  c4_<M>    one static-disorder realisation per bond-dimension class
            M in {32, 64, 96, 128} (the first realisation of that class):
            10 steps
  c3_cq, c4_96_cq, c4_128_cq
            the same runs with the shifted Cholesky QR of the oracle in
            place of Householder QR (10 / 6 steps): a second valid oracle
            trajectory, whose distance from the first measures how much the
            trajectory amplifies the choice of QR (the GPU factors the
            larger site tensors by shifted Cholesky QR)
  c5        217-site chain, M = 256, dt = 1 fs: the first step
  lz_<name> Krylov propagator exp(z H) x at the full local sizes of the
            M = 128 and M = 256 chains (H[i] and the bond operator):
            sampled output entries, the output norm and the Krylov dimension

Observables follow the oracle's conventions: populations <psi|n_m|psi> (not
divided by the norm), norm <psi|psi>, energy <psi|H'|psi> of the shifted
operator H' = H - shift (the constant is stored separately).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from inputs import chain_sites, workload, WORKLOADS  # noqa: E402
from inputs.fmo import ENSEMBLE, ensemble_bond, ensemble_members  # noqa: E402
from inputs.randt import random_complex, random_hermitian_env, random_mpo_like  # noqa: E402
from oracle import model, mps as om, ps  # noqa: E402
from oracle.krylov import expm_lanczos  # noqa: E402


def _observe(m, Ws, sites, n_e):
    return (om.norm2(m), om.expectation_mpo(m, Ws).real, om.site_populations(m, sites, n_e))


def _run_chain(p, sites, raw, tau, nsteps, kmax, record_every=1, log=None, save=None, qr=om.qr_pos):
    """Oracle TDVP-PS run; observables at step 0 and every record_every steps.
    save(partial results) is called after every recorded step, so a long
    run leaves a usable prefix if it is stopped.  qr: the QR of eq:QR."""
    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(raw, qr=qr)
    R = om.build_right_envs(m, Ws)
    steps, norms, energies, pops, ks = [], [], [], [], []

    def rec(s):
        nrm, e, pp = _observe(m, Ws, sites, p.n_e)
        steps.append(s)
        norms.append(nrm)
        energies.append(e)
        pops.append(pp)

    rec(0)
    t0 = time.time()
    for s in range(1, nsteps + 1):
        stats = {}
        m, R, _ = ps.ps_step(m, Ws, R, tau, kmax=kmax, stats=stats, qr=qr)
        ks.append(np.mean(stats["k"]))
        if s % record_every == 0 or s == nsteps:
            rec(s)
            if save:
                save(dict(steps=np.array(steps), norm=np.array(norms), energy=np.array(energies),
                          pops=np.array(pops), krylov_mean=np.array(ks)))
        if log:
            log(f"step {s}/{nsteps}  P0 {pops[-1][0]:.12f}  {time.time() - t0:.0f} s")
    return dict(steps=np.array(steps), norm=np.array(norms), energy=np.array(energies),
                pops=np.array(pops), krylov_mean=np.array(ks))


def _chain_target(name, wl, nsteps, realisation=None, qr=om.qr_pos):
    if realisation is None:
        w = dict(WORKLOADS[wl])
        p, sites, _, _, raw, _ = workload(wl)
        Mb = w["M"]
    else:   # a member of the static-disorder ensemble
        w = dict(ENSEMBLE)
        r, p, Mb, raw = ensemble_members(realisation + 1, w["seed"])[realisation]
        sites = chain_sites(p)
    tau = w["dt_fs"] * model.AU_PER_FS
    shift = model.shifted_terms(p, sites)[4]
    meta = dict(target=name, workload=wl, realisation=realisation, M=Mb, eta=w.get("eta", 0.0),
                phi_seed=w.get("phi_seed", 1), dt_fs=w["dt_fs"], kmax=w.get("kdim", 20),
                nsteps=nsteps, shift=shift, energy="shifted <psi|H'|psi>",
                qr="householder" if qr is om.qr_pos else "shifted cholesky qr3",
                made_by="tests/golden/make_goldens.py (oracle only)")
    out = _run_chain(p, sites, raw, tau, nsteps, w.get("kdim", 20),
                     log=lambda s: print(name, s, flush=True),
                     save=lambda part: _write(name, part, dict(meta, complete=False)), qr=qr)
    return out, dict(meta, complete=True)


# Local problems at the full sizes of the large chains: (Ml, d, Mr, Wl, Wr, z, seed).
# W = None marks the bond operator of eq:tdvp2_D (d = 1, Wl = Wr).
LZ_CASES = {
    "lz_m128": (128, 8, 128, 9, 9, -1.0j, 101),
    "lz_m256": (256, 10, 256, 9, 9, -1.0j, 102),
    "lz_bond256": (256, 1, 256, 9, 9, 1.0j, 103),
}
LZ_NSAMPLE = 4096


def lz_inputs(case):
    """Seeded operator and vector of a full-size Krylov case (shared with the
    GPU test): Hermitian environments, a Hermitian block-sparse MPO site
    (None for the bond operator) and a random start vector."""
    Ml, d, Mr, Wl, Wr, z, seed = LZ_CASES[case]
    L = random_hermitian_env(Ml, Wl, seed)
    R = random_hermitian_env(Mr, Wr, seed + 1)
    if d == 1:
        W = None
        x = random_complex((Ml, Mr), seed + 3)
    else:
        W0 = random_mpo_like(Wl, d, Wr, seed + 2, density=0.4)
        W = 0.5 * (W0 + np.conj(np.transpose(W0, (0, 2, 1, 3))))
        x = random_complex((Ml, d, Mr), seed + 3)
    return L, W, R, x, z


def lz_operator(L, W, R):
    """The oracle's operator of a Krylov case: H[i] (eq:tdvp1_H) or, for
    W = None, the bond operator (eq:tdvp2_D)."""
    if W is None:
        return lambda v: om.bond_op(L, R, v)
    return lambda v: om.heff(L, W, R, v)


def _lz_target(case):
    L, W, R, x, z = lz_inputs(case)
    # operator scale: |H x| = |x| for the start vector, so the propagator is
    # a moderate rotation (the GPU test scales L by the stored factor)
    s = np.linalg.norm(x) / np.linalg.norm(lz_operator(L, W, R)(x))
    L = L * s
    info = {}
    t0 = time.time()
    y = expm_lanczos(lz_operator(L, W, R), x, z, kmax=20, info=info)
    rng = np.random.default_rng(LZ_CASES[case][-1] + 17)
    idx = rng.integers(0, y.size, size=LZ_NSAMPLE)
    out = dict(scale=np.array(s), idx=idx, y=y.reshape(-1)[idx], ynorm=np.array(np.linalg.norm(y)),
               yabsmax=np.array(np.abs(y).max()), k=np.array(info["k"]))
    meta = dict(target=case, shape=list(LZ_CASES[case][:5]), z=str(LZ_CASES[case][5]), kmax=20,
                seconds=time.time() - t0, made_by="tests/golden/make_goldens.py (oracle only)")
    return out, meta


def c4_realisation(M):
    """The first disorder realisation of the 64-member ensemble with bond dimension M."""
    for r in range(64):
        if ensemble_bond(0, r) == M:
            return r
    raise ValueError(M)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("target")
    args = ap.parse_args()
    t = args.target
    if t == "c2":
        out, meta = _chain_target(t, "fmo7x10x8_M32", 500)
    elif t == "c3":
        out, meta = _chain_target(t, "fmo7x10x8_M128", 50)
    elif t == "c3_cq":
        out, meta = _chain_target(t, "fmo7x10x8_M128", 10, qr=om.qr_cholesky3)
    elif t.startswith("c4_") and t.endswith("_cq"):
        M = int(t[3:-3])
        out, meta = _chain_target(t, "ensemble", 6, realisation=c4_realisation(M), qr=om.qr_cholesky3)
    elif t.startswith("c4_"):
        M = int(t[3:])
        out, meta = _chain_target(t, "ensemble", 10, realisation=c4_realisation(M))
    elif t == "c5":
        out, meta = _chain_target(t, "fmo7x30x10_M256", 1)
    elif t in LZ_CASES:
        out, meta = _lz_target(t)
    else:
        raise SystemExit(f"unknown target {t}")
    print("wrote", _write(t, out, meta), flush=True)


def _write(target, out, meta):
    path = os.path.join(HERE, f"{target}.npz")
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, meta=np.array(json.dumps(meta)), **out)
    os.replace(tmp, path)
    return path


if __name__ == "__main__":
    main()
