"""What the trained network gains over the method without it.

The committed weights (trained by `python -m paper_2210_15668_amd.learn train` on
snapshots of the plain solver, seeds < 10000) start the Newton-multigrid solve of the
128 x 128 x 64 MFISM stack on held-out states (seeds >= 10000).  The plain method starts a
cold solve from phi = 0 (Step 0); the learned start must reach the same root (multigrid to
the same tolerance judges it) in fewer V-cycles, and an untrained network of the same
shape must not (the gain comes from the training).
"""
import os
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_15668_amd import ferrox
    ferrox.lib()
    return ferrox


def cold_cycles(fx, net, spec, seeds, vs):
    s = fx.Stack(spec, W.random_P(spec, seeds[0]))
    zeros = np.zeros((spec.nz, spec.ny, spec.nx))
    plain, learned, diffs = [], [], []
    for seed, v in zip(seeds, vs):
        P0 = W.random_P(spec, seed)
        s.set(fx.FIELD_P, P0)
        s.set(fx.FIELD_PHI, zeros)
        plain.append(s.poisson_solve(v).cycles)
        phi_plain = s.get(fx.FIELD_PHI)
        learned.append(net.learned_solve(s, v).cycles)
        phi_l = s.get(fx.FIELD_PHI)
        diffs.append(np.linalg.norm(phi_l - phi_plain) / np.linalg.norm(phi_plain))
    s.close()
    return np.array(plain), np.array(learned), max(diffs)


def test_trained_network_saves_cycles_on_held_out_cold_starts(fx):
    from paper_2210_15668_amd import learn
    spec = learn.spec_c4()
    kb, kt = spec.device_range()
    seeds = list(range(learn.TEST_SEED0 + 1, learn.TEST_SEED0 + 9))
    vs = list(np.random.default_rng(learn.TEST_SEED0).uniform(-2, 2, len(seeds)))
    net = fx.UNet(spec.nx, spec.ny, kt - kb)
    net.set_params(np.load(learn.WEIGHTS))
    plain, learned, diff = cold_cycles(fx, net, spec, seeds, vs)
    net.set_params(learn.init_params(7))
    _, untrained, diff_u = cold_cycles(fx, net, spec, seeds, vs)
    net.close()
    say(f"  cold start V-cycles: plain {plain.mean():.2f}, trained {learned.mean():.2f}, "
        f"untrained {untrained.mean():.2f}; max rel phi difference {diff:.1e} / {diff_u:.1e}")
    assert diff <= 1e-8 and diff_u <= 1e-8           # the same root, judged by multigrid
    assert learned.mean() <= plain.mean() - 2.0
    assert learned.mean() < untrained.mean() - 2.0


def test_learned_start_at_gate_jumps_saves_wall_time(fx):
    """End to end under a stepped gate (jumps of 1 to 2 V every 10 steps, held-out P^0): the
    solves at the jumps take less wall time started from the network's prediction than
    started from phi^n, and so does the whole run; both reach the same trajectory
    (multigrid to 1e-10 judges)."""
    from paper_2210_15668_amd import learn
    spec = learn.spec_c4()
    kb, kt = spec.device_range()
    net = fx.UNet(spec.nx, spec.ny, kt - kb)
    net.set_params(np.load(learn.WEIGHTS))
    r = learn.evaluate_gate_steps(net, spec)
    net.close()
    for k in ("restart", "learned"):
        say(f"  {k}: {r[k]['cycles']} V-cycles ({r[k]['jump_cycles']} at {r[k]['jumps']} jumps), "
            f"{r[k]['ms']:.2f} ms ({r[k]['jump_ms']:.2f} ms at the jumps)")
    say(f"  rel phi learned vs restart {r['rel_l2_phi_learned_vs_restart']:.1e}")
    assert r["learned"]["jump_cycles"] < r["restart"]["jump_cycles"]
    assert r["learned"]["jump_ms"] < r["restart"]["jump_ms"]
    assert r["learned"]["ms"] < r["restart"]["ms"]
    assert r["rel_l2_phi_learned_vs_restart"] <= 1e-7
