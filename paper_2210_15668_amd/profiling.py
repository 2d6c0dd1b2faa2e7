"""Turn rocprofv3 output into the short text summaries kept under profiles/.

Run on the GPU host from the repository root (each rocprofv3 call on its own); the
first, unprofiled bench run stores the tuned launch shapes in TUNE, so that the profiled
runs use the same shapes without the tuner's own timing launches:

  python3 bench.py --tune-cache TUNE
  rocprofv3 --kernel-trace --stats -d OUT/trace -o run -- python3 bench.py --no-batch --no-learned --no-variants --no-cpu-baseline --tune-cache TUNE
  rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o run -- python3 bench.py --steps 20 --no-mixed --no-batch --no-learned --no-cpu-baseline --no-variants --tune-cache TUNE
  rocprofv3 --pmc WRITE_SIZE -d OUT/write -o run -- python3 bench.py --steps 20 --no-mixed --no-batch --no-learned --no-cpu-baseline --no-variants --tune-cache TUNE
  rocprofv3 --pmc FETCH_SIZE -d OUT/cfetch -o run -- python3 -m paper_2210_15668_amd.profiling copy
  rocprofv3 --pmc WRITE_SIZE -d OUT/cwrite -o run -- python3 -m paper_2210_15668_amd.profiling copy
  python3 -m paper_2210_15668_amd.profiling stats OUT/trace
  python3 -m paper_2210_15668_amd.profiling traffic OUT

`copy` runs one plain device-to-device copy of 1 GiB (larger than the 256 MB
last-level cache, so every byte crosses HBM): FETCH_SIZE and WRITE_SIZE of that
dispatch, divided by 1 GiB, are the factors that turn the counters into bytes.

The learned start's network, per layer (forward passes of the committed weights on a
held-out state of the 128x128x64 MFISM stack):

  rocprofv3 --kernel-trace --stats -d OUT/unet -o run -- python3 -m paper_2210_15668_amd.profiling unet 20
  python3 -m paper_2210_15668_amd.profiling unet_layers OUT/unet

The V-cycle with and without the blocked smoothing of the small levels (FERROX_TB; the
same arithmetic either way): `steps N` runs Step 0, 10 untimed steps and N timed steps of
the 256x256x128 MFISM stack (FP64, or mixed with a second argument `mixed`) and prints
steps/s; `per_step OUT N` sums a kernel trace per time step (N steps in the trace):

  FERROX_TB=0 rocprofv3 --kernel-trace -d OUT/tb0 -o run -- python3 -m paper_2210_15668_amd.profiling steps 110
  FERROX_TB=1 rocprofv3 --kernel-trace -d OUT/tb1 -o run -- python3 -m paper_2210_15668_amd.profiling steps 110
  python3 -m paper_2210_15668_amd.profiling per_step OUT/tb0 120
  python3 -m paper_2210_15668_amd.profiling per_step OUT/tb1 120

Measured HBM bytes and instruction counts per launch of every kernel of a time step
(FETCH_SIZE / WRITE_SIZE calibrated by the copy runs above, in OUT/cfetch and OUT/cwrite):

  rocprofv3 --pmc FETCH_SIZE -d OUT/kfetch -o run -- python3 -m paper_2210_15668_amd.profiling steps 30
  rocprofv3 --pmc WRITE_SIZE -d OUT/kwrite -o run -- python3 -m paper_2210_15668_amd.profiling steps 30
  rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 -d OUT/ksq -o run -- python3 -m paper_2210_15668_amd.profiling steps 20
  python3 -m paper_2210_15668_amd.profiling kernels OUT
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2210_15668_amd", "csrc", "fx_kernels.hip")
COPY_BYTES = 1 << 30
# The dominant kernel: the FP64 Gauss-Seidel half-sweep on the finest level.  Its
# launches (all variants: zero start, plain, folded Newton update; either register
# budget) are those covering the most cells: grid x planes per thread (the third
# template argument).
SMOOTH64 = ("k_smooth<double", "k_smooth_w8<double")


def _cells(name, grid):
    if not name.startswith(SMOOTH64):
        return 0
    args = name[name.index("<") + 1:name.index(">")].split(",")
    return grid * int(args[2])


def _finest(keys):
    top = max(_cells(*k) for k in keys)
    return [k for k in keys if top > 0 and _cells(*k) == top]


def _db(d):
    files = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no rocprofv3 database under {d}")
    return sqlite3.connect(files[0])


def _short(name):
    m = re.search(r"(k_\w+)(<[^(]*>)?", name or "")
    return (m.group(1) + (m.group(2) or "")) if m else (name or "")[:48]


def copy():
    import torch
    n = COPY_BYTES // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {COPY_BYTES} bytes", flush=True)


def _working(values):
    """The launches that did work: a light cycle's skipped sweeps still launch, and every
    block returns at once (a few us, next to no bytes), far below the median."""
    med = sorted(values)[len(values) // 2] if values else 0.0
    return [v for v in values if v >= 0.25 * med]


def stats(trace_dir):
    db = _db(trace_dir)
    rows = db.execute("select name, grid_x, duration from kernels").fetchall()
    agg = defaultdict(lambda: [0, 0.0])
    durs = defaultdict(list)
    for name, gx, d in rows:
        key = (_short(name), gx)
        agg[key][0] += 1
        agg[key][1] += d
        durs[key].append(d)
    tot = sum(v[1] for v in agg.values())
    fine = _finest(list(agg))
    if fine:
        allv = [d for k in fine for d in durs[k]]
        work = _working(allv)
        print(f"Dominant kernel (finest-level FP64 smoother, {', '.join(f'`{k[0]}`' for k in fine)}): "
              f"{len(allv)} launches, average {sum(allv) / len(allv) / 1e3:.2f} us; the {len(work)} that did work "
              f"(a light cycle leaves the others empty) average {sum(work) / len(work) / 1e3:.2f} us\n")
    print("| kernel | grid (threads) | calls | avg us | total ms | % |")
    print("|---|---|---|---|---|---|")
    for (k, gx), (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:24]:
        print(f"| `{k}` | {gx} | {c} | {t / c / 1e3:.2f} | {t / 1e6:.2f} | {100 * t / tot:.1f} |")


def _counter(d, counter):
    db = _db(d)
    rows = db.execute("select kernel_name, grid_size, counter_name, value from counters_collection").fetchall()
    out = defaultdict(list)
    for name, grid, cname, v in rows:
        if cname == counter:
            out[(_short(name), grid)].append(v)
    return out


def traffic(base):
    """Measured HBM bytes per launch of the finest-level FP64 smoother (all its variants,
    weighted by their launch counts in the counter run; the empty launches of light
    cycles left out, as the in-run probe leaves them out)."""
    cf = _counter(os.path.join(base, "cfetch"), "FETCH_SIZE")
    cw = _counter(os.path.join(base, "cwrite"), "WRITE_SIZE")
    big_f = max(max(v) for v in cf.values()) * 1024.0
    big_w = max(max(v) for v in cw.values()) * 1024.0
    f_fetch, f_write = big_f / COPY_BYTES, big_w / COPY_BYTES
    fe = _counter(os.path.join(base, "fetch"), "FETCH_SIZE")
    wr = _counter(os.path.join(base, "write"), "WRITE_SIZE")
    fine = _finest(list(fe))
    fvals = _working([v for k in fine for v in fe[k]])
    wvals = _working([v for k in fine for v in wr.get(k, [])])
    fetch = sum(fvals) * 1024.0 / f_fetch / len(fvals)
    write = sum(wvals) * 1024.0 / f_write / max(1, len(wvals))
    with open(KERNEL_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out = {
        "kernel": "finest-level red/black Gauss-Seidel half-sweep (FP64), all variants",
        "variants": {f"{k[0]} grid {k[1]}": len(fe[k]) for k in fine},
        "dispatches_with_work": len(fvals),
        "copy_calibration": {"bytes": COPY_BYTES, "fetch_factor": f_fetch, "write_factor": f_write},
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "per_launch_bytes": {"fp64": fetch + write},
        "kernel_src_sha256": sha,
    }
    print(json.dumps(out, indent=1))


# Launches of one forward pass in order: (name, input channels of real work, output
# channels, level).  The skip layers also write the pooled tensor of the next level, the
# last layer applies the head.
UNET_LAUNCHES = [("e0a 3->16", 3, 16, 0), ("e0b 16->16 (+ 2x2x2 pooling)", 16, 16, 0),
                 ("e1a 16->32", 16, 32, 1), ("e1b 32->32 (+ 2x2x2 pooling)", 32, 32, 1),
                 ("b2a 32->64", 32, 64, 2), ("b2b 64->64, in 0..31", 32, 64, 2),
                 ("b2b 64->64, in 32..63", 32, 64, 2), ("d1a 96->32, upsampled 64", 64, 32, 1),
                 ("d1a 96->32, skip 32", 32, 32, 1), ("d1b 32->32", 32, 32, 1), ("d0a 48->16", 48, 16, 0),
                 ("d0b 16->16 (+ 1x1x1 head)", 16, 16, 0)]


def unet(reps):
    """reps forward passes (after three untimed ones) of the trained network."""
    import numpy as np
    import torch
    from paper_2210_15668_amd import ferrox, learn
    from paper_2210_15668_amd import workloads as W
    spec = learn.spec_c4()
    kb, kt = spec.device_range()
    net = ferrox.UNet(spec.nx, spec.ny, kt - kb)
    net.set_params(np.load(learn.WEIGHTS))
    st = ferrox.Stack(spec, W.random_P(spec, learn.TEST_SEED0 + 1))
    net.input_from_stack(st, 1.0)
    for _ in range(3):
        net.forward(copy=False)
    torch.cuda.synchronize()
    for _ in range(reps):
        net.forward(copy=False)
    torch.cuda.synchronize()
    st.close()
    net.close()
    print(f"{reps} forward passes of {spec.nx}x{spec.ny}x{kt - kb}", flush=True)


def unet_layers(trace_dir):
    """Median duration of each launch of a forward pass, with its real FLOP (multiply-adds
    counted as 2) and matrix-core rate."""
    from paper_2210_15668_amd import learn
    spec = learn.spec_c4()
    kb, kt = spec.device_range()
    n0 = spec.nx * spec.ny * (kt - kb)
    db = _db(trace_dir)
    rows = db.execute("select name, start, end from kernels order by start").fetchall()
    conv = [(_short(n), (b - a) / 1e3) for n, a, b in rows if _short(n).startswith("k_convz")]
    m = len(UNET_LAUNCHES)
    passes = [conv[i:i + m] for i in range(0, len(conv) - m + 1, m)]
    passes = passes[3:]                        # the untimed passes first
    print(f"{len(passes)} forward passes of {spec.nx}x{spec.ny}x{kt - kb}; median per launch\n")
    print("| launch | kernel | us | GFLOP | TFLOP/s |")
    print("|---|---|---|---|---|")
    tot_us = tot_fl = 0.0
    for i, (lname, ci, co, lev) in enumerate(UNET_LAUNCHES):
        d = sorted(p[i][1] for p in passes)[len(passes) // 2]
        fl = 2.0 * 27 * ci * co * n0 / 8 ** lev
        tot_us += d
        tot_fl += fl
        rate = f"{fl / d / 1e6:.0f}"
        print(f"| {lname} | `{passes[0][i][0]}` | {d:.2f} | {fl / 1e9:.2f} | {rate} |")
    print(f"| forward pass | (sum of medians) | {tot_us:.1f} | {tot_fl / 1e9:.1f} | {tot_fl / tot_us / 1e6:.0f} "
          f"({tot_fl / tot_us / 1e6 / 2500:.3f} of 2.5 PFLOP/s) |")


def kernels(base):
    """Per kernel (name, grid), medians over its dispatches: calibrated HBM bytes fetched
    and written, and VALU instructions per wave (all, and FP64 add/mul/fma)."""
    cf = _counter(os.path.join(base, "cfetch"), "FETCH_SIZE")
    cw = _counter(os.path.join(base, "cwrite"), "WRITE_SIZE")
    f_fetch = max(max(v) for v in cf.values()) * 1024.0 / COPY_BYTES
    f_write = max(max(v) for v in cw.values()) * 1024.0 / COPY_BYTES
    fe = _counter(os.path.join(base, "kfetch"), "FETCH_SIZE")
    wr = _counter(os.path.join(base, "kwrite"), "WRITE_SIZE")
    sq = {c: _counter(os.path.join(base, "ksq"), c) for c in
          ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64")}
    med = lambda v: sorted(v)[len(v) // 2] if v else 0.0
    rows = []
    for k, v in fe.items():
        f = med(v) * 1024.0 / f_fetch
        w = med(wr.get(k, [])) * 1024.0 / f_write
        rows.append((k, len(v), f, w))
    print(f"Calibration: a 1 GiB copy reads FETCH_SIZE x {f_fetch:.3f} and WRITE_SIZE x {f_write:.3f} of its bytes.\n")
    print("| kernel | grid | dispatches | fetch MB | write MB | VALU instr. per wave | FP64 add+mul+fma per wave |")
    print("|---|---|---|---|---|---|---|")
    for k, n, f, w in sorted(rows, key=lambda r: -(r[2] + r[3]) * r[1])[:16]:
        waves = med(sq["SQ_WAVES"].get(k, []))
        valu = med(sq["SQ_INSTS_VALU"].get(k, [])) / waves if waves else float("nan")
        f64 = sum(med(sq[c].get(k, [])) for c in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                                                    "SQ_INSTS_VALU_FMA_F64")) / waves if waves else float("nan")
        print(f"| `{k[0]}` | {k[1]} | {n} | {f / 1e6:.1f} | {w / 1e6:.1f} | {valu:.0f} | {f64:.0f} |")


def steps(n, prec_name="fp64"):
    import time
    import torch
    from paper_2210_15668_amd import ferrox
    from paper_2210_15668_amd import workloads as W
    prec = W.PREC_MIXED if prec_name == "mixed" else W.PREC_FP64
    spec = W.mfism_large(prec)
    s = ferrox.Stack(spec, W.random_P(spec, 2), device="cuda:0")
    s.run_steps(10, W.DT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = s.run_steps(n, W.DT)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    modes = s.levels(), s.level_modes()
    s.close()
    print(json.dumps({"prec": prec_name, "steps": n, "steps_per_s": n / (t1 - t0),
                      "vcycles_per_step": info.total_cycles / n, "levels": modes[0], "level_modes": modes[1]}),
          flush=True)


def per_step(trace_dir, n):
    """Kernel time per time step: launches, summed durations and the span from the first
    start to the last end, and the kernels with the largest share."""
    db = _db(trace_dir)
    rows = db.execute("select name, grid_x, duration, start, end from kernels order by start").fetchall()
    agg = defaultdict(lambda: [0, 0.0])
    for name, gx, d, _, _ in rows:
        agg[(_short(name), gx)][0] += 1
        agg[(_short(name), gx)][1] += d
    tot = sum(v[1] for v in agg.values())
    span = rows[-1][4] - rows[0][3]
    print(f"{len(rows) / n:.1f} launches, {tot / 1e3 / n:.1f} us of kernel time and {span / 1e3 / n:.1f} us of span "
          f"per time step ({n} steps in the trace)\n")
    print("| kernel | grid (threads) | calls per step | avg us | us per step |")
    print("|---|---|---|---|---|")
    for (k, gx), (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:24]:
        print(f"| `{k}` | {gx} | {c / n:.2f} | {t / c / 1e3:.2f} | {t / 1e3 / n:.1f} |")


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else ""
    if cmd == "copy":
        copy()
    elif cmd == "stats":
        stats(sys.argv[2])
    elif cmd == "traffic":
        traffic(sys.argv[2])
    elif cmd == "unet":
        unet(int(sys.argv[2]) if len(sys.argv) > 2 else 20)
    elif cmd == "unet_layers":
        unet_layers(sys.argv[2])
    elif cmd == "steps":
        steps(int(sys.argv[2]), sys.argv[3] if len(sys.argv) > 3 else "fp64")
    elif cmd == "per_step":
        per_step(sys.argv[2], float(sys.argv[3]))
    elif cmd == "kernels":
        kernels(sys.argv[2])
    else:
        print(__doc__)
        sys.exit(1)
