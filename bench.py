#!/usr/bin/env python3
"""TDGL + Poisson time steps per second on the 256x256x128 MFISM stack (one MI355X).

Workload: 256 x 256 x 128 cells of 0.5 nm; top-down gate metal 4 | ferroelectric 48
(HZO-like Landau coefficients, eps 24, lambda = 3 nm surface condition) | SiO2 8
(eps 3.9) | p-Si 64 (eps 11.7, Na = 1e24 m^-3, Boltzmann carriers, ni = 1e16 m^-3,
300 K) | back metal 4; 1 V gate; seeded uniform random P in +-0.01 C/m^2 (seed 2).
A step is the forward-Euler TDGL update plus the nonlinear Poisson solve to
||r|| <= 1e-10 ||f||, all inside the HIP library.  Step 0 (the initial solve) and
the warm-up steps are outside the timed region; fields are resident in HBM.

Prints one JSON line: FP64 steps/s (headline), the mixed-precision variant, the
roofline of the dominant kernel (the finest-level Gauss-Seidel half-sweep, timed
by its own dispatch events inside the timed region) and the CPU oracle's rate on
a bounded sample of the same stack.  Beside them: the batch of 64 uneven instances, the
learned warm start, and the same stack with the predictor-corrector time scheme and with
Fermi-Dirac carriers, plus a recorded Q-V sweep of the 3D MFIM of the Results.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "smooth_fine_mfism256_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2210_15668_amd", "csrc", "fx_kernels.hip")


def kernel_src_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(prec):
    """HBM bytes per launch of the dominant kernel from the committed counter runs,
    or None when the kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256") != kernel_src_hash():
        return None
    v = t.get("per_launch_bytes", {}).get(prec)
    return float(v) if v is not None else None


def run_gpu(prec_name, steps, warmup, tune=True, tune_cache=None):
    import torch
    from paper_2210_15668_amd import ferrox
    from paper_2210_15668_amd import workloads as W
    prec = W.PREC_FP64 if prec_name == "fp64" else W.PREC_MIXED
    spec = W.mfism_large(prec)
    P0 = W.random_P(spec, 2)
    s = ferrox.Stack(spec, P0, device="cuda:0")          # Step 0, untimed
    tuned = None
    if tune:                                             # launch-shape search, untimed
        ti = s.autotune(tune_cache)
        tuned = {"levels": ti.levels, "configs_timed": ti.configs_timed,
                 "half_sweep_us_default": ti.default_us, "half_sweep_us_tuned": ti.tuned_us,
                 "shapes": [dict(zip(("tile_x", "planes_per_thread", "waves8"), s.tune_config(l)))
                            for l in range(ti.levels)]}
    if warmup:
        s.run_steps(warmup, W.DT)
    torch.cuda.synchronize()
    # every 7th finest-level smoother launch of the timed region is timed by its own
    # dispatch events (timing every launch would slow the region by a few per cent);
    # 7 is prime to the 8 such launches of a V-cycle, so all variants are sampled
    s.probe(ferrox.PROBE_SMOOTH_FINE, max_launches=min(4096, max(64, steps * 2)), stride=7)
    t0 = time.perf_counter()
    info = s.run_steps(steps, W.DT)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches, nbytes = s.probe_read()
    s.probe(ferrox.PROBE_OFF)
    elapsed = t1 - t0
    out = {
        "steps_per_s": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "vcycles_per_step": info.total_cycles / max(1, steps),
        "last_rel_residual": info.last_res_rel,
        "probe_ms": ms, "probe_launches": launches, "probe_bytes": nbytes, "autotune": tuned,
    }
    out["phi"] = s.phi.detach().cpu().numpy()
    s.close()
    return out


def run_batch64(prec_name, steps, warmup, tune=True, tune_cache=None):
    """The 64 uneven MFIM instances advanced together (one launch per kernel for all of
    them, graph replay): time steps of the whole batch per second."""
    import torch
    from paper_2210_15668_amd import ferrox
    from paper_2210_15668_amd import workloads as W
    prec = W.PREC_FP64 if prec_name == "fp64" else W.PREC_MIXED
    inst = W.batch_instances(64)
    specs = [sp.copy(prec=prec) for sp, _ in inst]
    b = ferrox.Batch(specs, [P for _, P in inst], device="cuda:0")      # Step 0, untimed
    b.set_launch(ferrox.LAUNCH_GRAPH)
    ti = b.autotune(tune_cache) if tune else None
    if warmup:
        b.run(warmup, W.DT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = b.run(steps, W.DT)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    cells = sum(sp.ncell for sp in specs)
    return {"batch_steps_per_s": steps / dt, "instance_steps_per_s": 64 * steps / dt,
            "cells_total": cells, "vcycles_per_step_mean": sum(i.total_cycles for i in info) / (64.0 * steps),
            "vcycles_per_step_max": max(i.max_cycles_step for i in info),
            "autotune_half_sweep_us": None if ti is None else [ti.default_us, ti.tuned_us]}


def run_learned():
    """The learned warm start on the 128 x 128 x 64 MFISM stack with the committed trained
    weights, against plain multigrid on held-out states (both solved to 1e-10): cold starts,
    gate jumps and the time loop, plus the network's inference rate on the matrix cores."""
    import numpy as np
    from paper_2210_15668_amd import ferrox, learn
    spec = learn.spec_c4()
    kb, kt = spec.device_range()
    net = ferrox.UNet(spec.nx, spec.ny, kt - kb)
    net.set_params(np.load(learn.WEIGHTS))
    res = learn.evaluate(net, spec, n_cold=8, n_steps=50)
    res["inference"] = learn.inference_rate(net)
    net.close()
    res["workload"] = "MFISM 128x128x64 (metal 2 | FE 24 | SiO2 4 | p-Si 32 | metal 2), held-out seeds >= 10000"
    return res


def run_variants(steps):
    """The same 256 x 256 x 128 stack with the predictor-corrector (two solves per step)
    and with Fermi-Dirac carriers, and a recorded Q-V sweep of the 3D MFIM (Results)."""
    import torch
    from paper_2210_15668_amd import ferrox, sweep
    from paper_2210_15668_amd import workloads as W
    out = {}
    for name, spec in (("predictor_corrector", W.mfism_large().copy(time_order=2)),
                       ("fermi_dirac", W.mfism_large().copy(carriers=W.CARRIERS_FD))):
        s = ferrox.Stack(spec, W.random_P(spec, 2), device="cuda:0")
        s.run_steps(10, W.DT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.run_steps(steps, W.DT)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        out[name] = {"steps_per_s": steps / dt, "vcycles_per_step": info.total_cycles / steps, "steps": steps}
    spec = W.mfim_fig3()
    period = 4000
    r = sweep.run_sweep(spec, W.random_P(spec, 1, amp=0.01), 1000, 4.0, period)
    out["qv_sweep"] = {"workload": "3D MFIM 64x64x20 (5 nm FE / 4 nm Al2O3), +-4 V triangle, dt 4e-13 s, "
                                   "Q and V_fe recorded every step", "steps": r["steps"],
                       "steps_per_s": r["steps"] / r["seconds"], "vcycles_per_step": r["cycles"] / r["steps"]}
    return out


def cpu_baseline(sample_steps):
    """The oracle, as it stands, on the same z-stack with a 64 x 64 footprint (1/16 of
    the cells): Step 0 untimed, then `sample_steps` timed steps at the same tolerance;
    the rate is scaled by the cell ratio to the 256 x 256 x 128 workload."""
    import oracle
    from paper_2210_15668_amd import workloads as W
    full = W.mfism_large()
    spec = W.shrink_lateral(full, 64, 64)
    P0 = W.random_P(spec, 2)
    phi0, _ = oracle.solve(spec, P0, tol=full.tol_rel)
    t0 = time.perf_counter()
    oracle.run(spec, P0, sample_steps, W.DT, tol=full.tol_rel, phi0=phi0, init=False)
    dt = time.perf_counter() - t0
    ratio = (spec.nx * spec.ny) / (full.nx * full.ny)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sample_steps / dt * ratio, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample_steps} steps of the same stack on a 64x64 footprint (1/16 of the cells), "
                      f"{dt:.1f} s, rate scaled by the cell ratio; Step 0 untimed"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default smoother launch shapes")
    ap.add_argument("--tune-cache", default=None,
                    help="file of tuned launch shapes: read if it holds this workload, else written")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the predictor-corrector, Fermi-Dirac and Q-V lines")
    ap.add_argument("--batch-steps", type=int, default=500)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import oracle  # noqa: F401  (only for the cpu_baseline leg)

    r64 = run_gpu("fp64", args.steps, args.warmup, not args.no_tune, args.tune_cache)
    mixed = None
    if not args.no_mixed:
        rmx = run_gpu("mixed", args.steps, args.warmup, not args.no_tune, args.tune_cache)
        diff = float(np.linalg.norm(rmx["phi"] - r64["phi"]) / np.linalg.norm(r64["phi"]))
        mixed = {"value": rmx["steps_per_s"], "ms_per_step": rmx["ms_per_step"],
                 "vcycles_per_step": rmx["vcycles_per_step"], "dtype": "f32 multigrid in f64 defect correction",
                 "rel_l2_phi_vs_fp64_after_steps": diff,
                 "smoother_GBs": rmx["probe_bytes"] / (rmx["probe_ms"] * 1e-3) / 1e9 if rmx["probe_ms"] else None}
    avg_us = 1e3 * r64["probe_ms"] / max(1, r64["probe_launches"])
    per_launch = r64["probe_bytes"] / max(1, r64["probe_launches"])
    achieved = per_launch / (avg_us * 1e-6) / 1e9 if avg_us > 0 else 0.0
    traffic = measured_traffic("fp64")
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_smooth / k_smooth_w8 <double, ...> (finest-level red/black Gauss-Seidel half-sweep, FP64, all variants; launches a light cycle leaves empty are not counted)",
                "avg_launch_us": avg_us, "algorithmic_bytes_per_launch": per_launch,
                "launches_timed": r64["probe_launches"]}
    batch = None
    if not args.no_batch:
        b64 = run_batch64("fp64", args.batch_steps, 5, not args.no_tune, args.tune_cache)
        bmx = run_batch64("mixed", args.batch_steps, 5, not args.no_tune, args.tune_cache)
        batch = {"workload": "64 uneven MFIM instances: x, y in {32, 48, 64, 96}, z in {32, 48}, FE 16..32 / DE 4, "
                             "gates uniform in [-2, 2] V (seeds 100..163)",
                 "launch": "one launch per kernel for all instances, graph replay", "steps": args.batch_steps,
                 "fp64": b64, "mixed": bmx}
    learned = None if args.no_learned else run_learned()
    variants = None if args.no_variants else run_variants(100)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_sample_steps)
    line = {
        "metric": "TDGL+Poisson steps/s at 1e-10 residual, 256\u00b2\u00d7128 MFISM; plain MG vs learned",
        "value": r64["steps_per_s"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r64["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "MFISM 256x256x128 (metal 4 | FE 48 | SiO2 8 | p-Si 64 | metal 4), "
                               "Boltzmann carriers, dt 1e-13 s, 1 V gate, ||r||/||f|| <= 1e-10",
                   "solver": "Newton-multigrid V(2,2), extrapolated warm start",
                   "vcycles_per_step": r64["vcycles_per_step"],
                   "autotune": r64["autotune"],
                   "last_rel_residual": r64["last_rel_residual"]},
        "mixed_precision": mixed,
        "batch64": batch,
        "learned": learned,
        "variants": variants,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": "paper: ~15x node-by-node GPU vs multicore (4x A100 vs 32 Haswell cores, NERSC); "
                         "context only",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
