"""TDVP-PS throughput on one MI355X.

A step is one full symmetric TDVP-PS time step of a chain (left-to-right
and right-to-left sweeps: forward Lanczos solves, QR gauge shifts,
environment updates, backward bond solves, centre moves) followed by the
observables (norm, energy, populations); inputs are resident in HBM before
the timed region starts.

Default workload: the static-disorder ensemble -- 64 realisations of the
77-site chain (7 electronic sites x 10 modes x 8 levels), site energies
perturbed by N(0, 100 cm^-1), bond dimensions drawn from {32, 64, 96, 128},
dt = 2 fs, Krylov dimension 20, contractions in FP32 with FP64 Krylov, small
exponential and QR; ``value`` counts realisation-steps per second.  Its FP64
twin runs outside the timed region and states the mixed-mode error.
``--workload fmo7x10x8_M32`` (etc.) times one chain instead;
``--scheme mu-cmf`` / ``mu-vmf`` times TDVP-MU on such a chain (bond
dimension <= 64, FP64): a step is one constant-mean-field step of length
dt, or the variable-mean-field integration over dt.
Prints ONE JSON line (see the keys below).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense peaks; split-BF16 GEMMs do three bf16 products per real
# product, so their effective peak is the bf16 one over three
PEAK = {"fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "bf16x3_eff_tflops": 2500.0 / 3,
        "hbm_gbs": 8000.0}


def log(msg):
    """Progress of the benchmark's phases on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ensemble",
                    help="ensemble (default: the static-disorder ensemble) or a single-chain workload name")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "bf16x3"],
                    help="default: fp32 for the ensemble, fp64 for a single chain")
    ap.add_argument("--grouped", action="store_true",
                    help="ensemble: time the grouped launches (one launch sequence per Krylov solve for "
                         "every class) instead of one batched ensemble per class on its own stream")
    ap.add_argument("--alt-steps", type=int, default=2,
                    help="ensemble: steps of the other launch mode, timed after the main run")
    ap.add_argument("--twin-steps", type=int, default=5,
                    help="steps of the FP64 twin of a mixed-precision ensemble (outside the timed region)")
    ap.add_argument("--kmax", type=int, default=20)
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one (no step graph)")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-class-timing", action="store_true",
                    help="skip the per-kernel-class timing steps (for counter runs)")
    ap.add_argument("--realisations", type=int, default=64)
    ap.add_argument("--no-fused", action="store_true",
                    help="general multi-kernel Lanczos step everywhere (tdvp_set_fused(ctx, 0))")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="time candidate GEMM tile shapes of new problem keys in the first (warm-up) "
                         "step (tdvp_set_autotune); auto: on where the tiled GEMMs carry the "
                         "contractions (bond dimension > 64, the ensemble), off where the fused "
                         "small-bond step does (measured: no gain there)")
    ap.add_argument("--scheme", default="ps", choices=["ps", "ps2", "mu-cmf", "mu-vmf"],
                    help="single chain: TDVP-PS (default), two-site TDVP-PS (FP64, pairs up to 64 "
                         "wide), or TDVP-MU with constant or variable mean field (tolerances rtol "
                         "1e-5, atol 1e-8, eps 1e-10)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM counters)")
    return ap.parse_args()


def cpu_baseline(name, nsteps):
    """The oracle (plain numpy FP64, untuned) on a bounded sample of the same
    workload: nsteps steps at all host threads, one step at one thread."""
    from inputs import workload
    from oracle import model

    p, sites, phys, dims, raw, w = workload(name)
    tau = w["dt_fs"] * model.AU_PER_FS
    total, used = 0.0, 1
    for _ in range(nsteps):
        t, used = _oracle_step_seconds(p, sites, raw, tau)
        total += t
    t1, _ = _oracle_step_seconds(p, sites, raw, tau, threads=1)
    return {"value": nsteps / total, "unit": "steps/s", "cores": used, "kind": "oracle",
            "sample": f"{nsteps} first step(s) of {name} incl. populations, numpy FP64, at {used} "
                      f"threads; one step at 1 thread: {t1:.2f} s",
            "single_thread_steps_per_s": 1.0 / t1, **_cpu_info()}


# Kernel classes that are dense complex contractions (MFMA roof); the others
# are priced against HBM bandwidth.
MFMA_CLASSES = ("gemm", "gemm_heff", "lz_fused")
# the classes that carry H[i] x and the bond operator (H_eff TFLOP/s)
HEFF_CLASSES = ("gemm_heff", "lz_fused")
KERNEL_OF_CLASS = {"gemm": "cgemm_kernel", "gemm_heff": "cgemm_kernel", "lz_fused": "heff_small_kernel",
                   "lz_update": "lz_update_kernel",
                   "lz_dots": "lz_dots_kernel", "lz_ends": "lz_finish_kernel", "qr": "qr_reg_kernel",
                   "wapply": "wapply_kernel"}


DTYPE_OF = {0: "c128", 1: "c64 contractions / c128 Krylov+QR",
            2: "c64 (split-bf16 MFMA GEMMs) contractions / c128 Krylov+QR"}


# Timed launches of the contraction classes (GEMM, MPO pass, fused Lanczos
# step) run this many times back to back between their events, so the event
# time per launch is the kernel plus the gap between queued kernels, as
# rocprofv3 sees it, rather than one eager dispatch each.
TIMING_REPS = 4


def autotune_on(args):
    if args.autotune != "auto":
        return args.autotune == "on"
    if args.workload == "ensemble":
        return True
    from inputs import WORKLOADS
    return WORKLOADS[args.workload]["M"] > 64


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when there is none for this workload or the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_1907_12044_amd", "csrc", rec.get("source", ""))
    try:
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if digest != rec.get("source_sha256"):
        return None
    ent = rec.get("kernels", {}).get(f"{workload}/{precision}/{kernel}")
    return None if ent is None else ent.get("bytes_per_launch")


def roofline(prof, prec, ms_per_step, workload=None, precision=None):
    """Roofline entry for the kernel class with the largest time per step,
    from the event-timed class step: algorithmic FLOP (contractions) or bytes
    (the rest) per launch over the average launch time."""
    from paper_1907_12044_amd import tdvp
    if not prof:
        return None, None
    heff_flop = sum(prof[k]["flop"] for k in HEFF_CLASSES if k in prof)
    heff_tflops = heff_flop / (ms_per_step * 1e-3) / 1e12
    dom = max(prof, key=lambda k: prof[k]["ms_per_step"])
    d = prof[dom]
    t = d["ms_per_step"] * 1e-3
    if dom in MFMA_CLASSES:
        if prec == tdvp.FP64:
            peak = PEAK["fp64_mfma_tflops"]
        elif prec == tdvp.BF16X3 and dom == "gemm":
            peak = PEAK["bf16x3_eff_tflops"]
        else:
            peak = PEAK["fp32_mfma_tflops"]
        roof = {"bound": "mfma", "achieved": d["flop"] / t / 1e12, "peak": peak, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": d["bytes"] / t / 1e9, "peak": PEAK["hbm_gbs"], "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(KERNEL_OF_CLASS.get(dom, dom), workload, precision)
    roof["kernel"] = KERNEL_OF_CLASS.get(dom, dom)
    roof["launches_per_step"] = d["launches"]
    roof["timing_reps"] = TIMING_REPS if dom in ("gemm", "gemm_heff", "wapply", "lz_fused") else 1
    roof["avg_launch_us"] = 1e6 * t / max(d["launches"], 1)
    roof["per_launch"] = {"flop": d["flop"] / max(d["launches"], 1),
                          "bytes": d["bytes"] / max(d["launches"], 1)}
    return roof, heff_tflops


def _cpu_info():
    model_name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model_name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model_name}


def _oracle_step_seconds(p, sites, raw, tau, threads=None):
    """Wall time of one oracle TDVP-PS step (plain numpy FP64, untuned) of
    one chain, and the BLAS thread count it ran with."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import model, mps as om, ps

    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(raw)
    R = om.build_right_envs(m, Ws)
    with threadpool_limits(limits=threads):
        used = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
        t0 = time.perf_counter()
        m, R, _ = ps.ps_step(m, Ws, R, tau, kmax=20)
        om.site_populations(m, sites, p.n_e)
        dt = time.perf_counter() - t0
    return dt, used


def ensemble_cpu_baseline(members, sites, tau, class_flop):
    """The oracle on a bounded sample of the ensemble: one full step of the
    first M = 32 realisation (all host threads, then one thread) and of the
    first M = 64 realisation (all threads).  The per-step time of the
    M = 96 and 128 classes is extrapolated from the M = 64 step by the
    ratio of algorithmic contraction FLOP per step (the oracle takes minutes
    per step there); the ensemble rate is realisations over the summed
    per-class step times."""
    first = {}
    for r, p, M, raw in members:
        first.setdefault(M, (r, p, raw))
    t32, used = _oracle_step_seconds(first[32][1], sites, first[32][2], tau)
    t32_1, _ = _oracle_step_seconds(first[32][1], sites, first[32][2], tau, threads=1)
    t64, _ = _oracle_step_seconds(first[64][1], sites, first[64][2], tau)
    per = {32: t32, 64: t64}
    for M in (96, 128):
        per[M] = t64 * class_flop[M] / class_flop[64]
    counts = {}
    for _, _, M, _ in members:
        counts[M] = counts.get(M, 0) + 1
    total = sum(counts[M] * per[M] for M in counts)
    info = _cpu_info()
    return {"value": len(members) / total, "unit": "realisation-steps/s", "cores": used, "kind": "oracle",
            "sample": (f"one oracle step of realisation {first[32][0]} (M=32): {t32:.2f} s at {used} "
                       f"threads, {t32_1:.2f} s at 1 thread; one step of realisation {first[64][0]} "
                       f"(M=64): {t64:.2f} s; M=96/128 steps extrapolated from M=64 by algorithmic FLOP "
                       f"({per[96]:.1f} s, {per[128]:.1f} s); value = {len(members)} realisations / "
                       f"sum over classes of count x step time"),
            "single_thread_m32_steps_per_s": 1.0 / t32_1, "all_threads_m32_steps_per_s": 1.0 / t32,
            **info}


def step_flops(params, sites, M, k):
    """Algorithmic FLOP of the contractions of one PS step (structural MPO
    nonzeros; every Krylov solve of dimension k): per site 2 (k F_heff +
    F_env), per bond 2 k F_bond (F_heff = F_env = 8 [W_l M_l^2 d M_r +
    nnz(W) M_l M_r + W_r M_l d M_r^2], F_bond = 16 W M^3)."""
    import numpy as np
    from inputs import bond_dims
    from paper_1907_12044_amd import tdvp
    Ws, wb, _ = tdvp.fmo_model(params, sites)
    phys = [s_[3] for s_ in sites]
    mb = bond_dims(phys, M)
    n = len(sites)
    f = 0.0
    for i in range(n):
        Ml, d, Mr = mb[i], phys[i], mb[i + 1]
        nnz = int(np.count_nonzero(Ws[i]))
        fh = 8.0 * (wb[i] * Ml * Ml * d * Mr + nnz * Ml * Mr + wb[i + 1] * Ml * d * Mr * Mr)
        f += 2.0 * (k * fh + fh)
        if i < n - 1:
            f += 2.0 * k * 16.0 * wb[i + 1] * Mr ** 3
    return f


def ensemble_main(args):
    """The static-disorder ensemble: realisations of the 77-site chain with
    bond dimensions from {32, 64, 96, 128}, all advanced together (one
    ensemble per bond-dimension class, every kernel covering its class in
    one launch, classes on separate streams).  Timed in the requested
    (mixed) precision; an FP64 twin of the same ensemble runs outside the
    timed region to state the mixed-mode error and the FP64 rate."""
    import numpy as np
    import torch
    from inputs import chain_sites
    from inputs.fmo import ENSEMBLE, ensemble_members
    from paper_1907_12044_amd import tdvp

    nreal = args.realisations
    prec = {"fp64": tdvp.FP64, "fp32": tdvp.FP32, "bf16x3": tdvp.BF16X3}[args.precision]
    members = ensemble_members(nreal, ENSEMBLE["seed"])
    sites = chain_sites(members[0][1])
    tau = ENSEMBLE["dt_fs"] * tdvp.AU_PER_FS

    def build(pr, grouped=args.grouped):
        return tdvp.DisorderEnsemble(members, sites, 0, pr, kmax=args.kmax, tol=args.tol,
                                     graph=not args.eager, fused=not args.no_fused,
                                     autotune=autotune_on(args), grouped=grouped)

    ens = build(prec)
    torch.cuda.synchronize()
    log(f"ensemble of {nreal} built ({args.precision})")
    hist = [ens.observe_host()]          # observables after 0, 1, 2, ... steps
    for w in range(args.warmup):
        ens.step(tau, 1)
        hist.append(ens.observe_host())
        log(f"warm-up step {w + 1} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ens.step(tau, 1)
        hist.append(ens.observe_host())
        log(f"timed step {k + 1} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / max(args.steps, 1)

    prof = {}
    if not args.no_class_timing:
        for c_, _ in ens.contexts():
            tdvp.profile_reps(c_, TIMING_REPS)
        for name, cls in tdvp.PROF_CLASSES.items():
            acc = {"ms_per_step": 0.0, "launches": 0, "flop": 0.0, "bytes": 0.0}
            for c_, _ in ens.contexts():
                tdvp.profile(c_, cls)
            ens.step(tau, 1)
            for c_, _ in ens.contexts():
                ms_, n_, f_, b_ = tdvp.profile_read(c_)
                tdvp.profile(c_, 0)
                acc["ms_per_step"] += ms_
                acc["launches"] += n_
                acc["flop"] += f_
                acc["bytes"] += b_
            prof[name] = acc
            log(f"class timing {name} done")
    # algorithmic contraction FLOP of one step per bond-dimension class
    # (Krylov dimension kmax in every solve), for the CPU-baseline scaling
    class_flop = {M: step_flops(members[[m[2] for m in members].index(M)][1], sites, M, args.kmax)
                  for M in sorted({m[2] for m in members})}
    roof, heff_tflops = roofline(prof, prec, ms, f"ensemble{nreal}", args.precision)
    del ens
    torch.cuda.empty_cache()

    # the other launch mode, same precision, a few steps after one warm-up
    alt = {}
    if args.alt_steps > 0:
        ea = build(prec, grouped=not args.grouped)
        ea.step(tau, 1)
        ea.synchronize()
        ta = time.perf_counter()
        ea.step(tau, args.alt_steps)
        ea.observe_host()
        ta = time.perf_counter() - ta
        alt = {"launch_mode": "grouped" if not args.grouped else "per-class streams", "steps": args.alt_steps,
               "realisation_steps_per_s": nreal * args.alt_steps / ta, "ms_per_step": 1e3 * ta / args.alt_steps}
        log(f"other launch mode: {alt['realisation_steps_per_s']:.2f} realisation-steps/s")
        del ea
        torch.cuda.empty_cache()

    # FP64 twin: same members from t = 0, outside the timed region
    twin = {}
    if prec != tdvp.FP64 and args.twin_steps > 0:
        nt = min(args.twin_steps, len(hist) - 1)
        e64 = build(tdvp.FP64)
        e64.step(tau, 1)                  # first step: autotuning, graph capture
        torch.cuda.synchronize()
        log("FP64 twin: first step done")
        t1 = time.perf_counter()
        if nt > 1:
            e64.step(tau, nt - 1)
        o64 = e64.observe_host()
        t64 = time.perf_counter() - t1
        om_ = hist[nt]
        dP = np.abs(om_[:, 2:] - o64[:, 2:]).max()
        dn = np.abs(om_[:, 0] - o64[:, 0]).max()
        dE = np.abs(om_[:, 1] - o64[:, 1]).max()
        twin = {"steps_compared": nt, "max_abs_dpop": float(dP), "max_abs_dnorm": float(dn),
                "max_abs_denergy_hartree": float(dE),
                "max_abs_denergy_cm-1": float(dE / tdvp.HARTREE_PER_CM),
                "fp64_realisation_steps_per_s": (nreal * (nt - 1) / t64) if nt > 1 else None,
                "pop_error_within_1e-5": bool(dP <= 1e-5)}
        del e64
        torch.cuda.empty_cache()

    pops = hist[-1][:, 2:]
    prod = np.zeros(pops.shape[1])
    prod[0] = 1.0                     # exciton on electronic site 1, vibrational vacuum
    t0_dev = float(np.abs(hist[0][:, 2:] - prod[None, :]).max())
    counts = {}
    for _, _, M, _ in members:
        counts[M] = counts.get(M, 0) + 1
    line = {
        "metric": "TDVP-PS steps/s + H_eff TFLOP/s, mixed/batched vs FP64 at <=1e-5 pop error",
        "value": nreal * 1e3 / ms, "unit": "realisation-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_OF[prec],
        "data": "synthetic",
        "config": {"workload": f"fmo7x10x8_disorder_ensemble{nreal}", "sites": len(sites),
                   "classes": {str(M): counts[M] for M in sorted(counts)}, "dt_fs": ENSEMBLE["dt_fs"],
                   "precision": args.precision, "kmax": args.kmax, "autotune": autotune_on(args),
                   "graph": not args.eager,
                   "launch_mode": "grouped" if args.grouped else "per-class streams",
                   "initial_state_eta": ENSEMBLE["eta"],
                   # largest |P_m(0) - P_m(product state)| over the realisations
                   "t0_max_population_deviation": t0_dev},
        "ensemble_steps_per_s": 1e3 / ms,
        "heff_tflops": heff_tflops,
        "class_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in prof.items()},
        "roofline": roof,
        "fp64_twin": twin,
        "other_launch_mode": alt,
        "population_sum_range": [float(pops.sum(1).min()), float(pops.sum(1).max())],
    }
    if not args.no_cpu_baseline:
        if set(class_flop) >= {32, 64, 96, 128}:
            log("oracle timing (cpu_baseline)")
            line["cpu_baseline"] = ensemble_cpu_baseline(members, sites, tau, class_flop)
    print(json.dumps(line), flush=True)


def cpu_baseline_ps2(name):
    """The oracle's two-site step (plain numpy FP64, untuned) on the same
    workload: two steps at all host threads."""
    from threadpoolctl import threadpool_info
    from inputs import workload
    from oracle import model, mps as om, ps2

    p, sites, phys, dims, raw, w = workload(name)
    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(raw)
    R = om.build_right_envs(m, Ws)
    tau = w["dt_fs"] * model.AU_PER_FS
    t0 = time.perf_counter()
    for _ in range(2):
        m, R, _ = ps2.ps2_step(m, Ws, R, tau)
    dt = (time.perf_counter() - t0) / 2
    threads = max((t.get("num_threads", 1) for t in threadpool_info()), default=1)
    return {"value": 1.0 / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"two oracle two-site steps of {name}: {dt:.2f} s per step", **_cpu_info()}


def mu_main(args):
    """TDVP-MU on one chain: steps of length dt, the MPS left-canonicalised on
    the device first; the host takes every Runge-Kutta step decision."""
    import numpy as np
    import torch
    from inputs import workload
    from paper_1907_12044_amd import tdvp

    if args.precision != "fp64":
        log("TDVP-MU runs in FP64 only")
        sys.exit(2)
    p, sites, phys, dims, raw, w = workload(args.workload)
    run = tdvp.MuRun(p, sites, raw, 0, canonicalize=True)
    tau = w["dt_fs"] * tdvp.AU_PER_FS
    tol = dict(eps=1e-10, rtol=1e-5, atol=1e-8)
    if args.scheme == "mu-cmf":
        def step():
            return run.cmf_step(tau, 1, kmax=args.kmax, tol=args.tol, **tol)
    else:
        def step():
            return run.evolve(tau, **tol)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = [0, 0, 0]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        stats = [a + b for a, b in zip(stats, st)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / max(args.steps, 1)
    m = run.mps_numpy()
    gauge = 0.0
    for A in m[:-1]:
        X = A.reshape(-1, A.shape[2])
        gauge = max(gauge, float(np.abs(X.conj().T @ X - np.eye(X.shape[1])).max()))
    name = {"mu-cmf": "TDVP-MU (CMF)", "mu-vmf": "TDVP-MU (VMF)"}[args.scheme]
    line = {
        "metric": f"{name} steps/s",
        "value": 1e3 / ms_per_step,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "scheme": args.scheme, "sites": len(sites),
                   "bond_dim": w["M"], "dt_fs": w["dt_fs"], "kmax": args.kmax, **tol},
        "rk_steps_per_step": stats[0] / max(args.steps, 1),
        "rk_rejected_per_step": stats[1] / max(args.steps, 1),
        "rhs_evals_per_step": stats[2] / max(args.steps, 1),
        "final_norm": float(np.linalg.norm(m[-1])),
        "final_gauge_error": gauge,
        "roofline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent disorder realisations would be sharded one process per GPU", file=sys.stderr)
        sys.exit(2)
    if args.precision is None:
        args.precision = "fp32" if args.workload.startswith("ensemble") else "fp64"
    if args.workload.startswith("ensemble"):
        return ensemble_main(args)
    if args.scheme.startswith("mu"):
        return mu_main(args)
    import numpy as np
    import torch
    from inputs import workload
    from paper_1907_12044_amd import tdvp

    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p, sites, phys, dims, raw, w = workload(args.workload)
    prec = {"fp64": tdvp.FP64, "fp32": tdvp.FP32, "bf16x3": tdvp.BF16X3}[args.precision]
    two_site = args.scheme == "ps2"
    if two_site and prec != tdvp.FP64:
        log("two-site TDVP-PS runs in FP64 only")
        sys.exit(2)
    run = tdvp.PsRun(p, sites, raw, device=0, precision=prec, kmax=args.kmax, tol=args.tol,
                     graph=not args.eager and not two_site, fused=not args.no_fused,
                     autotune=autotune_on(args), two_site=two_site)
    tau = w["dt_fs"] * tdvp.AU_PER_FS
    nsolve = 4 * len(sites)
    with torch.cuda.stream(run.stream):
        klog = torch.zeros(nsolve, dtype=torch.int32, device="cuda:0")
        obs = torch.zeros((max(args.steps, 1), 2 + p.n_e), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        run.step(tau, 1)
        run.observe(obs[0])
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for s in range(args.steps):
        run.step(tau, 1)
        run.observe(obs[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / max(args.steps, 1)
    host_obs = obs.cpu().numpy()

    # one more step with a Krylov log, then one per kernel class with event timing
    tdvp.set_krylov_log(run.ctx, klog)
    run.step(tau, 1)
    tdvp.set_krylov_log(run.ctx, None)
    torch.cuda.synchronize()
    ks = klog.cpu().numpy()
    ks = ks[ks > 0]
    prof = {}
    if not args.no_class_timing:
        tdvp.profile_reps(run.ctx, TIMING_REPS)
        for name, cls in tdvp.PROF_CLASSES.items():
            tdvp.profile(run.ctx, cls)
            run.step(tau, 1)
            ms, n, f, b = tdvp.profile_read(run.ctx)
            tdvp.profile(run.ctx, 0)
            prof[name] = {"ms_per_step": ms, "launches": n, "flop": f, "bytes": b}
    roof, heff_tflops = roofline(prof, prec, ms_per_step, args.workload, args.precision)

    line = {
        "metric": ("two-site " if two_site else "") + "TDVP-PS steps/s (H_eff TFLOP/s alongside)",
        "value": 1e3 / ms_per_step,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_OF[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "sites": len(sites), "bond_dim": w["M"],
                   "mpo_bond_max": max(run.mpo.bond), "dt_fs": w["dt_fs"], "kmax": args.kmax,
                   "tol": args.tol, "precision": args.precision, "graph": not args.eager and not two_site,
                   "fused": not args.no_fused, "autotune": autotune_on(args)},
        "heff_tflops": heff_tflops,
        "krylov_mean": float(ks.mean()) if ks.size else None,
        "class_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in prof.items()},
        "roofline": roof,
        "final_populations": [float(x) for x in host_obs[-1, 2:]],
        "final_norm": float(host_obs[-1, 0]),
    }
    if two_site:
        line["config"]["scheme"] = "ps2"
        line["discarded_weight"] = float(run.discarded.cpu().numpy()[0])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = (cpu_baseline_ps2(args.workload) if two_site
                                else cpu_baseline(args.workload, args.cpu_steps))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
