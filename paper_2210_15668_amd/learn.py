"""Learned warm start: snapshot generation by the plain solver, training on the GPU, and the
comparison with plain multigrid.

Everything numerical runs in the HIP library through its C ABI (include/ferrox.h,
include/ferrox_unet.h): the plain FP64 Newton-multigrid solver produces the snapshots, the
library's BF16 MFMA kernels run the network forward and backward and apply Adam.  This
module only orders the calls.

Workload: the 128 x 128 x 64 MFISM stack (metal 2 | ferroelectric 24 | SiO2 4 | p-Si 32
| metal 2, cell 0.5 nm); the network works on its 60 device planes.
Snapshots (training): 2000 independent random P^0 fields (uniform +-0.01 C/m^2, seeds
0..1999) and 2000 states along 40 TDGL trajectories (seeds 5000..5039, a snapshot every 10
steps of dt = 1e-13 s, 50 per trajectory), each with a gate voltage uniform in [-2, 2] V
and phi solved by the plain solver to ||r|| <= 1e-10 ||f||.  Held-out evaluation seeds
are >= 10000.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time
from typing import Dict, List, Optional

import numpy as np

from . import ferrox
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "unet_mfism128.npy")
WEIGHTS_INFO = os.path.join(HERE, "weights", "unet_mfism128.json")

# (cin, cout) of the 3x3x3 convolutions in parameter order (include/ferrox_unet.h)
CONVS = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]
IN_CHANNELS = 3          # P, doping, V: the real inputs of the first layer (padded to 16 on the device)
TRAIN_SEEDS_IID = range(0, 2000)
TRAIN_SEEDS_TRAJ = range(5000, 5040)
TRAJ_SNAPSHOTS, TRAJ_STRIDE = 50, 10
TEST_SEED0 = 10000


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def spec_c4(prec: int = W.PREC_FP64) -> W.StackSpec:
    """The 128 x 128 x 64 MFISM stack: FE 24 / SiO2 4 / p-Si 32, metal 2 + 2."""
    return W.mfism_medium(prec)


def doping_planes(spec: W.StackSpec) -> np.ndarray:
    kb, kt = spec.device_range()
    sc = spec.plane_mat[kb:kt] == W.SC
    return np.where(sc, spec.plane_Nd[kb:kt] - spec.plane_Na[kb:kt], 0.0)


def init_params(seed: int) -> np.ndarray:
    """He-normal convolution weights (fan-in 27 cin), zero biases, a small random head."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CONVS:
        parts.append(rng.standard_normal(27 * co * ci) * math.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(16) * 0.0625)
    parts.append(np.zeros(1))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == ferrox.UNet.num_params()
    return theta


class Snapshots:
    """(P over the device planes, gate voltage, target) triples resident on the GPU."""

    def __init__(self, spec: W.StackSpec, n: int, device="cuda:0"):
        import torch
        kb, kt = spec.device_range()
        shape = (n, kt - kb, spec.ny, spec.nx)
        self.P = torch.empty(shape, dtype=torch.float32, device=device)
        self.T = torch.empty(shape, dtype=torch.float32, device=device)
        self.V = np.zeros(n)
        self.kind = [""] * n
        self.n = 0

    def add(self, stack: ferrox.Stack, net: ferrox.UNet, v: float, kind: str):
        kb, kt = stack.spec.device_range()
        self.P[self.n].copy_(stack.P[kb:kt])
        net.target_from_stack(stack, v, out=self.T[self.n])
        self.V[self.n] = v
        self.kind[self.n] = kind
        self.n += 1


def generate(spec: W.StackSpec, net: ferrox.UNet, iid_seeds, traj_seeds, traj_snapshots: int,
             traj_stride: int) -> Snapshots:
    rng = np.random.default_rng(12345)
    snaps = Snapshots(spec, len(iid_seeds) + len(traj_seeds) * traj_snapshots)
    st = ferrox.Stack(spec, W.random_P(spec, iid_seeds[0]))
    t0 = time.perf_counter()
    cycles = 0
    for q, seed in enumerate(iid_seeds):
        v = float(rng.uniform(-2.0, 2.0))
        st.set(ferrox.FIELD_P, W.random_P(spec, seed))
        cycles += st.poisson_solve(v).cycles
        snaps.add(st, net, v, "iid")
        if q % 250 == 0:
            log(f"[learn] iid snapshot {q}/{len(iid_seeds)} ({time.perf_counter() - t0:.1f} s)")
    for q, seed in enumerate(traj_seeds):
        v = float(rng.uniform(-2.0, 2.0))
        st.set(ferrox.FIELD_P, W.random_P(spec, seed))
        st.poisson_solve(v)
        for _ in range(traj_snapshots):
            st.run_steps(traj_stride, W.DT)
            snaps.add(st, net, v, "trajectory")
        log(f"[learn] trajectory {q + 1}/{len(traj_seeds)} ({time.perf_counter() - t0:.1f} s)")
    st.close()
    snaps.gen_seconds = time.perf_counter() - t0
    snaps.iid_cycles_mean = cycles / max(1, len(iid_seeds))
    return snaps


def train(net: ferrox.UNet, snaps: Snapshots, doping: np.ndarray, epochs: int, lr0: float, lr1: float,
          seed: int) -> Dict:
    rng = np.random.default_rng(seed)
    total = epochs * snaps.n
    step = 0
    t0 = time.perf_counter()
    curve = []
    run = []
    for ep in range(epochs):
        for idx in rng.permutation(snaps.n):
            lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * step / total))
            net.pack_input(snaps.P[idx], doping, snaps.V[idx])
            want = step % 50 == 0
            loss = net.train_step(snaps.T[idx], lr, want_loss=want)
            if want:
                run.append(loss)
            if step % 500 == 0:
                m = float(np.mean(run)) if run else float("nan")
                curve.append((step, m))
                log(f"[learn] step {step}/{total} epoch {ep} lr {lr:.2e} loss {m:.4e} "
                    f"({time.perf_counter() - t0:.1f} s)")
                run = []
            step += 1
    import torch
    torch.cuda.synchronize()
    return {"steps": step, "seconds": time.perf_counter() - t0, "curve": curve}


def validation_loss(net: ferrox.UNet, spec: W.StackSpec, doping: np.ndarray, seeds, v_values) -> float:
    """Mean loss on held-out independent P^0 fields (solved by the plain solver)."""
    import torch
    st = ferrox.Stack(spec, W.random_P(spec, seeds[0]))
    kb, kt = spec.device_range()
    tg = torch.empty((kt - kb, spec.ny, spec.nx), dtype=torch.float32, device="cuda:0")
    Pf = torch.empty_like(tg)
    losses = []
    for seed, v in zip(seeds, v_values):
        st.set(ferrox.FIELD_P, W.random_P(spec, seed))
        st.poisson_solve(v)
        net.target_from_stack(st, v, out=tg)
        Pf.copy_(st.P[kb:kt])
        net.pack_input(Pf, doping, v)
        out = net.forward()
        losses.append(float(torch.mean((out - tg) ** 2)))
    st.close()
    return float(np.mean(losses))


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def evaluate(net: ferrox.UNet, spec: W.StackSpec, n_cold: int = 16, n_steps: int = 100, seed0: int = TEST_SEED0) -> Dict:
    """Learned vs plain starting iterates on held-out states, both solved to the stack's
    tolerance by the same multigrid: cold starts (Step 0: phi = 0), gate-voltage jumps,
    and the time loop (plain: the extrapolated phi^n; learned: the prediction)."""
    rng = np.random.default_rng(seed0)
    st = ferrox.Stack(spec, W.random_P(spec, seed0))
    zeros = np.zeros((spec.nz, spec.ny, spec.nx))
    cold = {"plain_cycles": [], "learned_cycles": [], "plain_s": [], "learned_s": []}
    jump = {"plain_cycles": [], "learned_cycles": [], "plain_s": [], "learned_s": []}
    for q in range(n_cold):
        P0 = W.random_P(spec, seed0 + 1 + q)
        v = float(rng.uniform(-2.0, 2.0))
        st.set(ferrox.FIELD_P, P0)
        st.set(ferrox.FIELD_PHI, zeros)
        info, dt = timed(lambda: st.poisson_solve(v))
        cold["plain_cycles"].append(info.cycles)
        cold["plain_s"].append(dt)
        info, dt = timed(lambda: net.learned_solve(st, v))
        cold["learned_cycles"].append(info.cycles)
        cold["learned_s"].append(dt)
        # a jump of the gate by >= 1 V from the converged state
        v2 = float(np.clip(v + rng.choice([-1.0, 1.0]) * rng.uniform(1.0, 2.0), -2.0, 2.0))
        phi_v = st.get(ferrox.FIELD_PHI)
        info, dt = timed(lambda: st.poisson_solve(v2))
        jump["plain_cycles"].append(info.cycles)
        jump["plain_s"].append(dt)
        st.set(ferrox.FIELD_PHI, phi_v)
        info, dt = timed(lambda: net.learned_solve(st, v2))
        jump["learned_cycles"].append(info.cycles)
        jump["learned_s"].append(dt)
    st.close()
    # time loop from a held-out P^0 at a fixed gate
    v = 1.0
    P0 = W.random_P(spec, seed0 + 500)
    a = ferrox.Stack(spec.copy(v_top=v), P0)
    a.run_steps(10, W.DT)
    ri, dt_plain = timed(lambda: a.run_steps(n_steps, W.DT))
    b = ferrox.Stack(spec.copy(v_top=v), P0)
    b.run_steps(10, W.DT)

    def learned_loop():
        c = 0
        for _ in range(n_steps):
            b.tdgl_step(W.DT)
            c += net.learned_solve(b, v).cycles
        return c

    lc, dt_learned = timed(learned_loop)
    diff = float(np.linalg.norm(a.get(ferrox.FIELD_PHI) - b.get(ferrox.FIELD_PHI)) /
                 np.linalg.norm(a.get(ferrox.FIELD_PHI)))
    a.close()
    b.close()

    def summ(d):
        return {"plain_cycles_mean": float(np.mean(d["plain_cycles"])),
                "learned_cycles_mean": float(np.mean(d["learned_cycles"])),
                "cycles_saved_mean": float(np.mean(d["plain_cycles"]) - np.mean(d["learned_cycles"])),
                "plain_ms_mean": 1e3 * float(np.mean(d["plain_s"])),
                "learned_ms_mean": 1e3 * float(np.mean(d["learned_s"])),
                "n": len(d["plain_cycles"])}

    return {"cold_start": summ(cold), "voltage_jump": summ(jump),
            "gate_steps": evaluate_gate_steps(net, spec),
            "time_loop": {"steps": n_steps, "plain_vcycles_per_step": ri.total_cycles / n_steps,
                          "plain_steps_per_s": n_steps / dt_plain,
                          "learned_vcycles_per_step": lc / n_steps,
                          "learned_steps_per_s": n_steps / dt_learned,
                          "rel_l2_phi_learned_vs_plain": diff}}


def jump_steps(sched: np.ndarray, v0: float, thresh: float) -> List[int]:
    """Steps whose gate differs from the previous step's by more than thresh volts."""
    prev = np.concatenate([[v0], sched[:-1]])
    return [int(n) for n in np.nonzero(np.abs(sched - prev) > thresh)[0]]


def run_gate_schedule(stack: ferrox.Stack, n_steps: int, dt: float, sched: np.ndarray, policy: str,
                      net: Optional[ferrox.UNet] = None, thresh: float = 0.5) -> Dict:
    """n_steps time steps of the stack under a gate schedule (entry n for the solve producing
    phi^{n+1}).  Smooth stretches run through run_steps, whose solves start from the
    extrapolation in time.  At a step where the gate jumps by more than thresh (known from
    the schedule in advance) that extrapolation is no valid start (carried through a jump
    of 1.5 V it diverges), so the step runs Step 1a and then a solve from
      policy "restart": phi^n (the start the paper's Step 1b takes),
      policy "learned": the network's prediction for the new gate;
    multigrid to the same tolerance judges either start.  Returns the V-cycles, those of
    the jump steps alone and the wall time of the jump steps (device synchronised)."""
    import torch
    v0 = stack.spec.v_top
    jumps = jump_steps(sched, v0, thresh)
    cycles = jump_cycles = 0
    jump_s = 0.0
    n = 0
    for j in jumps + [n_steps]:
        if j > n:
            cycles += stack.run_steps(j - n, dt, sched[n:j]).total_cycles
            n = j
        if j < n_steps:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            stack.tdgl_step(dt)
            info = net.learned_solve(stack, float(sched[j])) if policy == "learned" else \
                stack.poisson_solve(float(sched[j]))
            torch.cuda.synchronize()
            jump_s += time.perf_counter() - t0
            cycles += info.cycles
            jump_cycles += info.cycles
            n = j + 1
    return {"cycles": cycles, "jump_cycles": jump_cycles, "jump_ms": 1e3 * jump_s, "steps": n_steps,
            "jumps": len(jumps)}


def gate_steps_schedule(n_steps: int = 120, seg: int = 10) -> np.ndarray:
    """A stepped gate: 1.0, -0.5, 1.5, 0.0, 1.0, -1.0 V, seg steps each (jumps of 1 to 2 V)."""
    levels = [1.0, -0.5, 1.5, 0.0, 1.0, -1.0]
    return np.array([levels[(n // seg) % len(levels)] for n in range(n_steps)])


def evaluate_gate_steps(net: ferrox.UNet, spec: W.StackSpec, n_steps: int = 120, seg: int = 10,
                        seed: int = TEST_SEED0 + 700, runs: int = 3) -> Dict:
    """End-to-end time steps under a stepped gate (held-out P^0): the solves at the jumps
    started from phi^n ("restart") or from the network ("learned"), the same 1e-10
    tolerance everywhere; per policy the fastest of `runs` runs."""
    sched = gate_steps_schedule(n_steps, seg)
    P0 = W.random_P(spec, seed)
    out = {"workload": f"{n_steps} steps, gate stepped every {seg} steps (1.0, -0.5, 1.5, 0.0, 1.0, -1.0 V), "
                       f"held-out P^0; the fastest of {runs} runs per policy"}
    net.forward()                                   # the network's kernels loaded before timing
    phis = {}
    for policy in ("restart", "learned"):
        best = None
        for _ in range(runs):
            st = ferrox.Stack(spec.copy(v_top=1.0), P0)
            st.run_steps(5, W.DT)                   # history before the first stretch
            r, dt_s = timed(lambda: run_gate_schedule(st, n_steps, W.DT, sched, policy, net))
            r["ms"] = 1e3 * dt_s
            r["steps_per_s"] = n_steps / dt_s
            phis[policy] = st.get(ferrox.FIELD_PHI)
            st.close()
            if best is None or r["ms"] < best["ms"]:
                best = r
        out[policy] = best
    ref = phis["restart"]
    out["rel_l2_phi_learned_vs_restart"] = float(np.linalg.norm(phis["learned"] - ref) / np.linalg.norm(ref))
    return out


def inference_rate(net: ferrox.UNet, reps: int = 20) -> Dict:
    """Forward passes per second on the current input (the output left in the workspace,
    as a learned solve uses it) and the matrix-core throughput they imply (multiply-adds of the 3x3x3 convolutions counted as 2 FLOP).  Only real work
    counts: the first layer has 3 input channels (P, doping, V), whatever width the
    kernel pads them to."""
    nz, ny, nx = net.shape
    n0 = nx * ny * nz
    flops = 0
    for q, (ci, co) in enumerate(CONVS):
        n = n0 if q in (0, 1, 8, 9) else (n0 // 8 if q in (2, 3, 6, 7) else n0 // 64)
        flops += 2 * 27 * (IN_CHANNELS if q == 0 else ci) * co * n
    for _ in range(3):
        net.forward(copy=False)
    _, dt = timed(lambda: [net.forward(copy=False) for _ in range(reps)])
    s = dt / reps
    return {"ms": 1e3 * s, "flop": flops, "tflops": flops / s / 1e12, "peak_tflops_bf16": 2500.0,
            "frac": flops / s / 1e12 / 2500.0}


def main(argv: Optional[List[str]] = None):
    import argparse
    ap = argparse.ArgumentParser(description="train / evaluate the learned warm start")
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--iid", type=int, default=len(TRAIN_SEEDS_IID))
    ap.add_argument("--traj", type=int, default=len(TRAIN_SEEDS_TRAJ))
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--weights", default=WEIGHTS)
    args = ap.parse_args(argv)
    spec = spec_c4()
    kb, kt = spec.device_range()
    doping = doping_planes(spec)
    if args.cmd == "train":
        net = ferrox.UNet(spec.nx, spec.ny, kt - kb, train=True)
        theta0 = init_params(7)
        net.set_params(theta0)
        snaps = generate(spec, net, list(TRAIN_SEEDS_IID)[:args.iid], list(TRAIN_SEEDS_TRAJ)[:args.traj],
                         TRAJ_SNAPSHOTS, TRAJ_STRIDE)
        log(f"[learn] {snaps.n} snapshots in {snaps.gen_seconds:.1f} s")
        val_seeds = list(range(TEST_SEED0 + 900, TEST_SEED0 + 916))
        val_v = list(np.random.default_rng(TEST_SEED0 + 900).uniform(-2, 2, len(val_seeds)))
        val0 = validation_loss(net, spec, doping, val_seeds, val_v)
        hist = train(net, snaps, doping, args.epochs, args.lr, args.lr * 0.01, seed=11)
        val1 = validation_loss(net, spec, doping, val_seeds, val_v)
        theta = net.get_params()
        os.makedirs(os.path.dirname(args.out), exist_ok=True)
        np.save(args.out, theta)
        info = {"workload": "MFISM 128x128x64 (metal 2 | FE 24 | SiO2 4 | p-Si 32 | metal 2)",
                "snapshots": snaps.n, "iid": args.iid, "trajectories": args.traj,
                "snapshot_generation_s": snaps.gen_seconds, "iid_plain_cycles_mean": snaps.iid_cycles_mean,
                "epochs": args.epochs, "lr": [args.lr, args.lr * 0.01], "train_steps": hist["steps"],
                "train_s": hist["seconds"], "train_step_ms": 1e3 * hist["seconds"] / max(1, hist["steps"]),
                "loss_curve": hist["curve"], "validation_loss_untrained": val0, "validation_loss_trained": val1}
        with open(WEIGHTS_INFO if args.out == WEIGHTS else args.out + ".json", "w") as f:
            json.dump(info, f, indent=1)
        log(f"[learn] validation loss {val0:.4e} -> {val1:.4e}")
        print(json.dumps({k: v for k, v in info.items() if k != "loss_curve"}), flush=True)
    else:
        net = ferrox.UNet(spec.nx, spec.ny, kt - kb)
        net.set_params(np.load(args.weights))
        res = evaluate(net, spec)
        res["inference"] = inference_rate(net)
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
