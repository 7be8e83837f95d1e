"""TDVP-PS throughput on one MI355X.

A step is one full symmetric TDVP-PS time step of the whole chain (left-to-
right and right-to-left sweeps: forward Lanczos solves, QR gauge shifts,
environment updates, backward bond solves, centre moves) followed by the
observables (norm, energy, populations) written to device memory; inputs
are resident in HBM before the timed region starts.

Default workload: 7 electronic sites x 10 modes x 8 levels (77 MPS sites),
bond dim 32, dt = 2 fs, complex128, Krylov dim 20.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fmo7x10x8_M32")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM counters)")
    return ap.parse_args()


def cpu_baseline(name, nsteps):
    """The oracle (plain numpy FP64, untuned) on a bounded sample of the same workload."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from inputs import workload
    from oracle import model, mps as om, ps

    p, sites, phys, dims, raw, w = workload(name)
    Ws, _ = model.mpo(p, sites)
    m = om.right_canonicalize(raw)
    R = om.build_right_envs(m, Ws)
    tau = w["dt_fs"] * model.AU_PER_FS
    t0 = time.perf_counter()
    for _ in range(nsteps):
        m, R, _ = ps.ps_step(m, Ws, R, tau, kmax=20)
        om.site_populations(m, sites, p.n_e)
    dt = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    return {"value": nsteps / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsteps} step(s) of {name} incl. populations, numpy FP64 "
                      f"({os.cpu_count()} host CPUs visible)"}


# Kernel classes that are dense complex contractions (MFMA roof); the others
# are priced against HBM bandwidth.
MFMA_CLASSES = ("gemm", "lz_fused")
KERNEL_OF_CLASS = {"gemm": "cgemm_kernel", "lz_fused": "heff_small_kernel", "lz_update": "lz_update_kernel",
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
    heff_flop = sum(prof[k]["flop"] for k in MFMA_CLASSES if k in prof)
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
    roof["timing_reps"] = TIMING_REPS if dom in ("gemm", "wapply", "lz_fused") else 1
    roof["avg_launch_us"] = 1e6 * t / max(d["launches"], 1)
    roof["per_launch"] = {"flop": d["flop"] / max(d["launches"], 1),
                          "bytes": d["bytes"] / max(d["launches"], 1)}
    return roof, heff_tflops


def ensemble_main(args):
    """64 static-disorder realisations, bond dims from {32, 64, 96, 128}: one
    PsEnsemble per bond-dimension class (every kernel covers the class in one
    launch), the classes on separate streams so they run concurrently."""
    import numpy as np
    import torch
    from inputs import draw_params, chain_sites, initial_mps_raw
    from inputs.fmo import ensemble_bond
    from paper_1907_12044_amd import tdvp

    nreal = args.realisations
    prec = {"fp64": tdvp.FP64, "fp32": tdvp.FP32, "bf16x3": tdvp.BF16X3}[args.precision]
    classes = {}
    for r in range(nreal):
        classes.setdefault(ensemble_bond(0, r), []).append(r)
    ens = []
    for M, rs in sorted(classes.items()):
        ps_ = [draw_params(7, 10, 8, seed=0, realisation=r) for r in rs]
        sites = chain_sites(ps_[0])
        raws = [initial_mps_raw(p, M, 1e-2, 1) for p in ps_]
        ens.append((M, rs, tdvp.PsEnsemble(ps_, sites, raws, 0, prec, kmax=args.kmax, tol=args.tol,
                                           graph=not args.eager, fused=not args.no_fused,
                                           autotune=autotune_on(args))))
    tau = 2.0 * tdvp.AU_PER_FS
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        for _, _, e in ens:
            e.step(tau, 1)
            e.observe()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for _, _, e in ens:
            e.step(tau, 1)
            e.observe()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / max(args.steps, 1)
    prof = {}
    if not args.no_class_timing:
        for _, _, e in ens:
            tdvp.profile_reps(e.ctx, TIMING_REPS)
        for name, cls in tdvp.PROF_CLASSES.items():
            acc = {"ms_per_step": 0.0, "launches": 0, "flop": 0.0, "bytes": 0.0}
            for _, _, e in ens:
                tdvp.profile(e.ctx, cls)
                e.step(tau, 1)
                ms_, n_, f_, b_ = tdvp.profile_read(e.ctx)
                tdvp.profile(e.ctx, 0)
                acc["ms_per_step"] += ms_
                acc["launches"] += n_
                acc["flop"] += f_
                acc["bytes"] += b_
            prof[name] = acc
    roof, heff_tflops = roofline(prof, prec, ms, f"ensemble{nreal}", args.precision)
    pops = np.concatenate([e.observe_host()[:, 2:] for _, _, e in ens])
    line = {
        "metric": "TDVP-PS ensemble steps/s (all realisations advanced one step)",
        "value": 1e3 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_OF[prec],
        "data": "synthetic",
        "config": {"workload": f"fmo7x10x8_ensemble{nreal}", "classes": {str(M): len(rs) for M, rs, _ in ens},
                   "precision": args.precision, "kmax": args.kmax, "autotune": autotune_on(args)},
        "realisation_steps_per_s": nreal * 1e3 / ms,
        "heff_tflops": heff_tflops,
        "class_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in prof.items()},
        "roofline": roof,
        "population_sum_range": [float(pops.sum(1).min()), float(pops.sum(1).max())],
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent disorder realisations would be sharded one process per GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload.startswith("ensemble"):
        return ensemble_main(args)
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
    run = tdvp.PsRun(p, sites, raw, device=0, precision=prec, kmax=args.kmax, tol=args.tol,
                     graph=not args.eager, fused=not args.no_fused, autotune=autotune_on(args))
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
        "metric": "TDVP-PS steps/s (H_eff TFLOP/s alongside)",
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
                   "tol": args.tol, "precision": args.precision, "graph": not args.eager,
                   "fused": not args.no_fused, "autotune": autotune_on(args)},
        "heff_tflops": heff_tflops,
        "krylov_mean": float(ks.mean()) if ks.size else None,
        "class_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in prof.items()},
        "roofline": roof,
        "final_populations": [float(x) for x in host_obs[-1, 2:]],
        "final_norm": float(host_obs[-1, 0]),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
