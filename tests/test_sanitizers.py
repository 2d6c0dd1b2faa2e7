"""CPU sanitizer tier: the oracle and the library's host-side planner built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on odd and degenerate shapes.

* oracle: Step 0, forward-Euler and predictor-corrector steps, residual norms, Poisson
  parts and Q-V on small stacks (odd sizes, a 1x1 column, 2D rows, metal-free, Fermi-Dirac);
* planner (host-only build of the HIP sources, no GPU): descriptor validation, the
  hierarchy, coarse-kernel LDS layout, launch planning and workspace layout of every
  stack and of all of them as one batch (the 64 uneven instances of the batched workload
  among them), plus descriptors that must be rejected; the sizes must equal the regular
  build's.
Any sanitizer report makes the driver exit non-zero.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
CSRC = os.path.join(ROOT, "paper_2210_15668_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def small_stacks():
    L = W.layered
    return [
        W.mfim_small(),
        L(12, 10, 19, [(W.FE, 7, W.EPS_FE, 0.0), (W.DE, 3, W.EPS_SIO2, 0.0), (W.SC, 5, W.EPS_SI, 1e24)],
          pbc=W.PBC_ZERO, v_top=0.6),
        L(1, 1, 40, [(W.FE, 9, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_AL2O3, 0.0), (W.SC, 20, W.EPS_SI, 1e24)], v_top=-0.8),
        L(6, 2, 7, [(W.FE, 3, W.EPS_FE, 0.0), (W.DE, 2, W.EPS_SIO2, 0.0)], v_top=0.3),
        L(16, 1, 32, [(W.FE, 16, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)], v_top=1.0),
        L(20, 1, 30, [(W.FE, 10, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0), (W.SC, 14, W.EPS_SI, 1e24)], v_top=0.9),
        L(9, 7, 23, [(W.FE, 17, W.EPS_FE, 0.0), (W.DE, 6, W.EPS_SIO2, 0.0)], pbc=W.PBC_FREE, v_top=1.7),
        W.mfism_fig4(8),
    ]


def planner_stacks():
    big = [W.mfism_large(), W.mfim_ramp(), W.mfism_medium(), W.shrink_lateral(W.mfism_large(), 64, 1),
           W.shrink_lateral(W.mfism_large(), 256, 1), W.convergence_mfism(64)]
    return small_stacks() + big + [sp for sp, _ in W.batch_instances(64)]


def write_list(path, specs):
    with open(path, "w") as f:
        for s in specs:
            f.write(f"{s.nx} {s.ny} {s.nz} {s.h!r} {s.pbc} {s.lam!r} {s.ni!r} {s.T!r} {s.v_top!r} {s.carriers}\n")
            for k in range(s.nz):
                f.write(f"{int(s.plane_mat[k])} {float(s.plane_eps_r[k])!r} {float(s.plane_Na[k])!r} "
                        f"{float(s.plane_Nd[k])!r}\n")


def run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


def san_env(leaks):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={1 if leaks else 0}:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    return env


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_san")
    run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
         "-fno-sanitize-recover=all", os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    lst = str(tmp_path / "stacks.txt")
    write_list(lst, small_stacks())
    out = run([exe, lst], env=san_env(True))
    lines = [l for l in out.splitlines() if l.startswith("stack")]
    assert len(lines) == len(small_stacks())
    for l in lines:
        assert "status 0" in l, l
        assert float(l.split("|r|/|f| ")[1].split()[0]) <= 1e-12, l


@pytest.mark.slow
def test_planner_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    objs = []
    for src in ("fx_stack.hip", "fx_kernels.hip", "fx_unet.hip", "fx_unet_conv.hip"):
        o = str(tmp_path / src.replace(".hip", ".o"))
        # the device code is built as usual; the sanitizers instrument the host code alone
        run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
             "-c", os.path.join(CSRC, src), "-o", o], timeout=900)
        objs.append(o)
    drv = str(tmp_path / "planner_driver.o")
    run([HIPCC, "--offload-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
         "-Xarch_host", "-fsanitize=address,undefined", "-c", os.path.join(SAN, "planner_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "planner_san")
    run([HIPCC, "--offload-arch=gfx950", "-g", "-Xarch_host", "-fsanitize=address,undefined", drv, *objs, "-o", exe])
    specs = planner_stacks()
    lst = str(tmp_path / "stacks.txt")
    write_list(lst, specs)
    out = run([exe, lst], env=san_env(False))
    # the same sizes as the regular library's planner
    from paper_2210_15668_amd import ferrox
    got = {}
    for l in out.splitlines():
        if l.startswith("stack") or l.startswith("batch prec"):
            key, val = l.rsplit(":", 1)
            got[key] = int(val)
    for prec in (0, 1):
        for order in (1, 2):
            sp = [s.copy(prec=prec, time_order=order) for s in specs]
            for i in (0, 3, 8, len(specs) - 1):
                assert got[f"stack {i} prec {prec} order {order}"] == ferrox.workspace_bytes(sp[i])
            assert got[f"batch prec {prec} order {order}"] == ferrox.batch_workspace_bytes(sp)
            assert all(got[f"stack {i} prec {prec} order {order}"] > 0 for i in range(len(specs)))
    assert "batch of 0: 0" in out
