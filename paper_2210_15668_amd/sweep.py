"""Q-V sweeps of a ferroelectric gate stack (Results, MFIM: the Q-V_fe and Q-V_app loops).

The stack relaxes at 0 V from a small random polarisation, then follows a triangular gate
wave; Q (interface charge density) and V_fe (average ferroelectric voltage) are recorded
after every time step on the device (run_steps_qv).  `loop_features` reads the last period's
rising and falling quarter-branches for the multidomain/single-domain switching voltages,
the width of the first-quadrant loop and the sign of dQ/dV_fe (negative capacitance) in the
multidomain state.

    python -m paper_2210_15668_amd.sweep --n 64 --vmax 4 --period 16000 --csv qv.csv
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Dict, Optional

import numpy as np

from . import ferrox as fx
from . import workloads as W


def run_sweep(spec: W.StackSpec, P0: np.ndarray, relax: int, v_max: float, period: int, periods: int = 1,
              dt: float = W.DT_TABLE1, launch: int = fx.LAUNCH_GRAPH) -> Dict[str, np.ndarray]:
    s = fx.Stack(spec, P0)
    s.set_launch(launch)
    if relax:
        s.run_steps(relax, dt, np.zeros(relax))
    n = period * periods
    v = W.triangle_schedule(n, v_max, period)
    t0 = time.perf_counter()
    info, Q, V = s.run_steps_qv(n, dt, v)
    el = time.perf_counter() - t0
    s.close()
    return {"v": v, "Q": Q, "V_fe": V, "seconds": el, "steps": n, "cycles": info.total_cycles}


def loop_features(v: np.ndarray, Q: np.ndarray, V_fe: np.ndarray, period: int) -> Dict[str, float]:
    """Features of the last period's first-quadrant loop (rising quarter 0 -> v_max, falling
    quarter v_max -> 0)."""
    base = len(v) - period
    q = period // 4
    up = slice(base, base + q)
    dn = slice(base + q, base + 2 * q)
    vu, Qu, Fu = v[up], Q[up], V_fe[up]
    vd, Qd, Fd = v[dn][::-1], Q[dn][::-1], V_fe[dn][::-1]
    # switching: the largest single-step drop of V_fe on the way up (into the single domain)
    # and the largest rise on the way down (back to the multidomain state)
    i_sd = int(np.argmin(np.diff(Fu)))
    i_md = int(np.argmin(np.diff(Fd)))
    grid = np.linspace(max(vu[0], vd[0]), min(vu[-1], vd[-1]), 200)
    width = np.interp(grid, vd, Qd) - np.interp(grid, vu, Qu)
    # multidomain part of the rising branch: below the switching voltage
    md = slice(0, max(i_sd - 1, 2))
    slope = np.polyfit(Fu[md], Qu[md], 1)[0] if i_sd > 3 else float("nan")
    return {
        "V_SD": float(0.5 * (vu[i_sd] + vu[i_sd + 1])),
        "V_MD": float(0.5 * (vd[i_md] + vd[i_md + 1])),
        "loop_max_dQ": float(width.max()),
        "Q_max": float(Q[base:].max()),
        "Q_at_0V_up": float(Qu[0]),
        "dQ_dVfe_multidomain": float(slope),
    }


def main(argv: Optional[list] = None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=64, help="lateral cells (64 = the paper's 32 nm)")
    ap.add_argument("--vmax", type=float, default=4.0)
    ap.add_argument("--period", type=int, default=16000, help="steps per triangle period")
    ap.add_argument("--periods", type=int, default=1)
    ap.add_argument("--relax", type=int, default=3000, help="steps at 0 V before the sweep")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--time-order", type=int, default=1)
    ap.add_argument("--csv", default=None, help="write step, V_app, Q, V_fe rows here")
    a = ap.parse_args(argv)
    spec = W.mfim_fig3(a.n).copy(time_order=a.time_order)
    P0 = W.random_P(spec, a.seed, amp=0.01)
    r = run_sweep(spec, P0, a.relax, a.vmax, a.period, a.periods)
    feat = loop_features(r["v"], r["Q"], r["V_fe"], a.period)
    feat.update(steps_per_s=r["steps"] / r["seconds"], cycles_per_step=r["cycles"] / r["steps"])
    print(json.dumps(feat))
    if a.csv:
        np.savetxt(a.csv, np.column_stack([np.arange(1, r["steps"] + 1), r["v"], r["Q"], r["V_fe"]]),
                   delimiter=",", header="step,V_app,Q,V_fe", comments="")


if __name__ == "__main__":
    main()
