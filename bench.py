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


def model_bytes_per_step(spec, vcycles, prec_name):
    """The one-touch byte model of a time step: the TDGL update reads P and phi and writes P
    (24 B per ferroelectric cell); each V(2,2) cycle moves about 149 B (FP64) or 114 B (FP32
    multigrid inside the FP64 defect correction) per device cell over all levels, residual
    and update included; the residual of the starting iterate reads phi and writes r (24 B,
    mixed 20 B per device cell)."""
    per_cycle, per_res = (149.0, 24.0) if prec_name == "fp64" else (114.0, 20.0)
    return 24.0 * spec.n_fe() + (vcycles * per_cycle + per_res) * spec.n_active()


def copy_bandwidth(nbytes=1 << 30, reps=20):
    """Device-to-device copy of a 1 GiB buffer: read + write bytes per second (GB/s)."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def whole_step(spec, r, prec_name, copy_gbs):
    b = model_bytes_per_step(spec, r["vcycles_per_step"], prec_name)
    gbs = b * r["steps_per_s"] / 1e9
    return {"model_bytes_per_step": b, "GBs": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS,
            "frac_of_measured_copy": gbs / copy_gbs if copy_gbs else None,
            "vcycles_per_step": r["vcycles_per_step"]}


def run_ramp(prec_name="fp64", nsteps=2000):
    """The 128 x 128 x 64 MFIM with its gate ramped 0 -> 1.5 V over 2000 steps, run in full:
    Step 0 untimed, then the 2000 steps timed."""
    import torch
    from paper_2210_15668_amd import ferrox
    from paper_2210_15668_amd import workloads as W
    spec = W.mfim_ramp().copy(prec=W.PREC_FP64 if prec_name == "fp64" else W.PREC_MIXED)
    vs = W.ramp_schedule(nsteps, 1.5, 2000)
    s = ferrox.Stack(spec, W.random_P(spec, 1), device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = s.run_steps(nsteps, W.DT, vs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    r = {"steps_per_s": nsteps / dt, "ms_per_step": 1e3 * dt / nsteps, "steps": nsteps,
         "vcycles_per_step": info.total_cycles / nsteps, "last_rel_residual": info.last_res_rel}
    return spec, r


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
    cores = oracle_threads()
    return {"value": sample_steps / dt * ratio, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{sample_steps} steps of the same stack on a 64x64 footprint (1/16 of the cells), "
                      f"{dt:.1f} s, rate scaled by the cell ratio; Step 0 untimed"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    """Threads the oracle's OpenMP loops use: OMP_NUM_THREADS, else the CPUs this process may run on."""
    v = os.environ.get("OMP_NUM_THREADS")
    if v and v.isdigit():
        return int(v)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_configs(path, which):
    """The oracle, as it stands, timed on the workloads in full (the 16x16x32 MFIM: Step 0 +
    100 steps; the 128x128x64 MFIM ramp: Step 0 + 2000 steps; the 64 uneven MFIM instances:
    Step 0 + 500 steps each) and on a stated subset of the 256x256x128 MFISM (Step 0 + 20
    steps), all at ||r|| <= 1e-10 ||f|| as on the GPU.  Writes a JSON summary to `path`
    after each workload and prints a progress line per workload (and per 100 steps)."""
    import numpy as np
    import oracle
    from paper_2210_15668_amd import workloads as W
    out = {"cpu_model": cpu_model(), "threads": oracle_threads(), "kind": "oracle",
           "tolerance": "||r|| <= 1e-10 ||f|| per solve", "workloads": {}}

    def save():
        with open(path, "w") as f:
            json.dump(out, f, indent=1)

    def timed_run(spec, P0, nsteps, sched, label, chunk=100):
        t0 = time.perf_counter()
        phi, _ = oracle.solve(spec, P0, tol=spec.tol_rel)
        t_step0 = time.perf_counter() - t0
        P = P0
        t1 = time.perf_counter()
        done = 0
        while done < nsteps:
            n = min(chunk, nsteps - done)
            vs = None if sched is None else sched[done:done + n]
            P, phi, _ = oracle.run(spec, P, n, W.DT, v_sched=vs, tol=spec.tol_rel, phi0=phi, init=False)
            done += n
            print(f"  {label}: {done}/{nsteps} steps, {time.perf_counter() - t1:.1f} s", flush=True)
        return t_step0, time.perf_counter() - t1

    if "c0" in which:
        spec = W.mfim_small()
        t0, ts = timed_run(spec, W.random_P(spec, 0), 100, None, "MFIM 16x16x32")
        out["workloads"]["mfim16_small"] = {"workload": "MFIM 16x16x32, 1 V, 100 steps (in full)",
                                            "step0_s": t0, "steps": 100, "steps_s": ts, "steps_per_s": 100 / ts}
        save()
    if "c1" in which:
        spec = W.mfim_ramp()
        vs = W.ramp_schedule(2000, 1.5, 2000)
        t0, ts = timed_run(spec, W.random_P(spec, 1), 2000, vs, "MFIM 128x128x64 ramp")
        out["workloads"]["mfim128_ramp"] = {"workload": "MFIM 128x128x64, gate ramp 0 -> 1.5 V over 2000 steps "
                                                        "(in full)", "step0_s": t0, "steps": 2000, "steps_s": ts,
                                            "steps_per_s": 2000 / ts}
        save()
    if "c2" in which:
        spec = W.mfism_large()
        t0, ts = timed_run(spec, W.random_P(spec, 2), 20, None, "MFISM 256x256x128", chunk=5)
        out["workloads"]["mfism256"] = {"workload": "MFISM 256x256x128, 1 V: Step 0 + 20 of the bench's 210 "
                                                    "steps (subset)", "step0_s": t0, "steps": 20, "steps_s": ts,
                                        "steps_per_s": 20 / ts}
        save()
    c3 = [w for w in which if w == "c3" or w.startswith("c3:")]
    if c3:
        # c3 or c3:a-b (instances a..b-1, so that the 64 can be timed in parts)
        lo, hi = (0, 64) if c3[0] == "c3" else tuple(int(x) for x in c3[0][3:].split("-"))
        t_all0 = t_all = 0.0
        per = []
        for q, (spec, P0) in enumerate(W.batch_instances(64)):
            if not lo <= q < hi:
                continue
            t0, ts = timed_run(spec, P0, 500, None, f"batch instance {q} {spec.nx}x{spec.ny}x{spec.nz}", chunk=250)
            t_all0 += t0
            t_all += ts
            per.append({"instance": q, "step0_s": t0, "steps_s": ts})
        out["workloads"][f"batch64_{lo}_{hi}"] = {
            "workload": f"instances {lo}..{hi - 1} of the 64 uneven MFIM instances, 500 steps each (in full), "
                        "one instance after another", "step0_s": t_all0, "steps": 500, "steps_s": t_all,
            "instances": per}
        save()
    return out


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
    ap.add_argument("--no-ramp", action="store_true", help="skip the 128x128x64 gate-ramp line")
    ap.add_argument("--oracle-configs", metavar="JSON", default=None,
                    help="only time the CPU oracle on the workloads in full (no GPU) and write JSON")
    ap.add_argument("--oracle-which", default="c0,c1,c2,c3",
                    help="workloads of --oracle-configs: c0 16x16x32, c1 128x128x64 ramp, c2 256^2x128 subset, "
                         "c3 batch of 64")
    args = ap.parse_args()
    if args.oracle_configs:
        oracle_configs(args.oracle_configs, set(args.oracle_which.split(",")))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import oracle  # noqa: F401  (only for the cpu_baseline leg)

    from paper_2210_15668_amd import workloads as W
    r64 = run_gpu("fp64", args.steps, args.warmup, not args.no_tune, args.tune_cache)
    copy_gbs = copy_bandwidth()
    spec_l = W.mfism_large()
    step64 = whole_step(spec_l, r64, "fp64", copy_gbs)
    mixed = None
    if not args.no_mixed:
        rmx = run_gpu("mixed", args.steps, args.warmup, not args.no_tune, args.tune_cache)
        diff = float(np.linalg.norm(rmx["phi"] - r64["phi"]) / np.linalg.norm(r64["phi"]))
        mixed = {"value": rmx["steps_per_s"], "ms_per_step": rmx["ms_per_step"],
                 "vcycles_per_step": rmx["vcycles_per_step"], "dtype": "f32 multigrid in f64 defect correction",
                 "rel_l2_phi_vs_fp64_after_steps": diff,
                 "smoother_GBs": rmx["probe_bytes"] / (rmx["probe_ms"] * 1e-3) / 1e9 if rmx["probe_ms"] else None,
                 "whole_step": whole_step(spec_l, rmx, "mixed", copy_gbs)}
    ramp = None
    if not args.no_ramp:
        spec_r, rr = run_ramp("fp64")
        rr["whole_step"] = whole_step(spec_r, rr, "fp64", copy_gbs)
        rr["workload"] = ("MFIM 128x128x64 (metal 8 | FE 40 | SiO2 8 | metal 8), gate ramped 0 -> 1.5 V over "
                          "2000 steps, FP64, ||r||/||f|| <= 1e-10, Step 0 untimed")
        ramp = rr
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
        "whole_step": step64,
        "copy_GBs_measured": copy_gbs,
        "mixed_precision": mixed,
        "mfim128_ramp": ramp,
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
