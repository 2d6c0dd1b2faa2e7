"""Batches of uneven stacks (one launch per kernel for all instances) against the oracle and
against the same instances run as stacks of their own.

No arithmetic crosses instances and every kernel computes a cell the same way whatever
else shares its launch, so an instance of a batch must reproduce its single-stack result
bitwise, in graph replay and in kernel-by-kernel launches alike.  Against the oracle the bar
is the single stack's: relative L2 <= 1e-10 for P and phi after N steps with both sides
solving to 1e-13.  The 64-instance workload (x, y in {32, 48, 64, 96}, z in {32, 48}) solves
to the production tolerance 1e-10; there every instance is checked through properties the
oracle evaluates independently: the oracle's residual of the GPU's phi for the GPU's P, and
the oracle's TDGL update of the GPU's state.
"""
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W
from parity_check import worst

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


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


# Uneven instances: split red/black and plainly stored levels (odd nx, odd ny), odd plane
# counts, semiconductor layers, every polarisation boundary condition.
MIX = [
    (16, 16, 32, [(W.FE, 16, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)], W.PBC_LAMBDA, 1.0),
    (24, 16, 30, [(W.FE, 12, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0), (W.SC, 8, W.EPS_SI, 1e24)],
     W.PBC_FREE, -0.7),
    (15, 16, 28, [(W.FE, 10, W.EPS_FE, 0.0), (W.DE, 3, W.EPS_AL2O3, 0.0)], W.PBC_ZERO, 0.5),
    (32, 32, 48, [(W.FE, 20, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)], W.PBC_LAMBDA, 1.5),
    (12, 10, 19, [(W.FE, 7, W.EPS_FE, 0.0), (W.DE, 3, W.EPS_SIO2, 0.0), (W.SC, 5, W.EPS_SI, 1e24)],
     W.PBC_ZERO, 0.6),
    (8, 8, 12, [(W.FE, 4, W.EPS_FE, 0.0), (W.DE, 2, W.EPS_SIO2, 0.0)], W.PBC_FREE, -1.2),
    (20, 9, 26, [(W.FE, 9, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0), (W.SC, 9, W.EPS_SI, 1e24)],
     W.PBC_LAMBDA, 0.9),
]


def mix_specs(prec, tol):
    """An odd lateral size stops the x-y coarsening at the finest level; multigrid then
    contracts slowly (about 0.7 per cycle for 20x9), so those instances get a larger cycle
    budget."""
    specs, Ps = [], []
    for q, (nx, ny, nz, layers, pbc, v) in enumerate(MIX):
        mc = 60 if nx % 2 == 0 and ny % 2 == 0 else 400
        sp = W.layered(nx, ny, nz, layers, pbc=pbc, v_top=v, tol_rel=tol, prec=prec, max_cycles=mc)
        specs.append(sp)
        Ps.append(W.random_P(sp, 40 + q, amp=0.05))
    return specs, Ps


def schedules(specs, nsteps):
    """Odd instances ramp their gate from v_top towards v_top + 0.4 V, even ones hold it."""
    out = []
    for q, sp in enumerate(specs):
        if q % 2:
            out.append(sp.v_top + 0.4 * np.arange(1, nsteps + 1) / nsteps)
        else:
            out.append(np.full(nsteps, sp.v_top))
    return out


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_batch_matches_oracle(fx, orc, prec):
    specs, Ps = mix_specs(prec, 1e-13)
    say(f"  batch of {len(specs)} uneven instances, prec={prec}")
    b = fx.Batch(specs, Ps)
    for q, sp in enumerate(specs):
        phi_o, _ = orc.solve(sp, Ps[q], tol=1e-13)
        assert worst(sp, b.get(q, fx.FIELD_PHI), phi_o) <= 1e-10, q
    n = 8
    vs = schedules(specs, n)
    info = b.run(n, W.DT, vs)
    for q, sp in enumerate(specs):
        assert info[q].status == fx.FX_OK and info[q].steps_done == n
        P_o, phi_o, _ = orc.run(sp, Ps[q], n, W.DT, v_sched=vs[q], tol=1e-13)
        rp, rf = worst(sp, b.get(q, fx.FIELD_P), P_o), worst(sp, b.get(q, fx.FIELD_PHI), phi_o)
        say(f"  inst {q} {sp.nx}x{sp.ny}x{sp.nz}: cycles/step {info[q].total_cycles / n:.2f} "
            f"relP {rp:.2e} relphi {rf:.2e}")
        assert rp <= 1e-10 and rf <= 1e-10, q


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_batch_equals_single_stacks(fx, prec):
    specs, Ps = mix_specs(prec, 1e-10)
    n = 10
    vs = schedules(specs, n)
    runs = {}
    for mode in (fx.LAUNCH_GRAPH, fx.LAUNCH_STREAM):
        b = fx.Batch(specs, Ps)
        b.set_launch(mode)
        info = b.run(4, W.DT, [v[:4] for v in vs])
        info2 = b.run(n - 4, W.DT, [v[4:] for v in vs])
        runs[mode] = ([b.get(q, fx.FIELD_P) for q in range(len(specs))],
                      [b.get(q, fx.FIELD_PHI) for q in range(len(specs))],
                      [i.total_cycles for i in info], [i.total_cycles for i in info2])
        b.close()
    for q in range(len(specs)):
        assert np.array_equal(runs[fx.LAUNCH_GRAPH][0][q], runs[fx.LAUNCH_STREAM][0][q]), q
        assert np.array_equal(runs[fx.LAUNCH_GRAPH][1][q], runs[fx.LAUNCH_STREAM][1][q]), q
    assert runs[fx.LAUNCH_GRAPH][2:] == runs[fx.LAUNCH_STREAM][2:]
    for q, sp in enumerate(specs):
        s = fx.Stack(sp, Ps[q])
        i1 = s.run_steps(4, W.DT, vs[q][:4])
        i2 = s.run_steps(n - 4, W.DT, vs[q][4:])
        assert (i1.total_cycles, i2.total_cycles) == (runs[fx.LAUNCH_GRAPH][2][q], runs[fx.LAUNCH_GRAPH][3][q])
        assert np.array_equal(s.get(fx.FIELD_P), runs[fx.LAUNCH_GRAPH][0][q]), q
        assert np.array_equal(s.get(fx.FIELD_PHI), runs[fx.LAUNCH_GRAPH][1][q]), q
        s.close()


def test_gate_to_zero_in_a_batch(fx):
    """A MOS stack (no ferroelectric) whose gate steps from 1 V to 0 V: from then on the
    right-hand side is exactly zero while the extrapolated start is not, so each such
    solve stops at its root phi = 0 (N(0) = 0) with every device cell exactly 0; an
    MFIM instance in the same launches still equals its own single-stack run bitwise."""
    mos = W.layered(32, 32, 24, [(W.DE, 4, W.EPS_SIO2, 0.0), (W.SC, 16, W.EPS_SI, 1e24)], v_top=1.0,
                    tol_rel=1e-10, ni=1.0e16, T=300.0)
    mfim = W.layered(32, 32, 32, [(W.FE, 16, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)], v_top=0.5,
                     tol_rel=1e-10)
    specs = [mos, mfim]
    Ps = [np.zeros((mos.nz, mos.ny, mos.nx)), W.random_P(mfim, 98, amp=0.05)]
    vs = [[1.0, 0.0, 0.0, 0.0], [0.5, 0.5, -0.5, -0.5]]
    b = fx.Batch(specs, Ps)
    info = b.run(4, W.DT, vs)
    assert all(i.status == fx.FX_OK and i.steps_done == 4 for i in info)
    dev = np.asarray(mos.plane_mat) != W.METAL
    phi0 = b.get(0, fx.FIELD_PHI)
    say(f"  MOS at 0 V: max |phi| on device planes {np.abs(phi0[dev]).max()}, last rel. residual "
        f"{info[0].last_res_rel}")
    assert np.all(phi0[dev] == 0.0) and info[0].last_res_rel == 0.0
    s = fx.Stack(mfim, Ps[1])
    s.run_steps(4, W.DT, vs[1])
    assert np.array_equal(s.get(fx.FIELD_P), b.get(1, fx.FIELD_P))
    assert np.array_equal(s.get(fx.FIELD_PHI), b.get(1, fx.FIELD_PHI))
    s.close()
    b.close()


def test_batch_failure_is_isolated(fx):
    """An instance that cannot converge stops with FX_ENOCONV; the others finish every step
    and still equal their single-stack results."""
    specs, Ps = mix_specs(W.PREC_FP64, 1e-10)
    bad = 2
    specs[bad] = specs[bad].copy(max_cycles=1, tol_rel=1e-14)
    b = fx.Batch(specs, Ps, check_init=False)
    assert b.init_status == fx.FX_ENOCONV
    info = b.run(5, W.DT, check=False)
    for q, sp in enumerate(specs):
        if q == bad:
            assert info[q].status == fx.FX_ENOCONV and info[q].steps_done == 0
            continue
        assert info[q].status == fx.FX_OK and info[q].steps_done == 5
        s = fx.Stack(sp, Ps[q])
        s.run_steps(5, W.DT)
        assert np.array_equal(s.get(fx.FIELD_PHI), b.get(q, fx.FIELD_PHI)), q
        s.close()
    with pytest.raises(fx.FerroxError):
        b.run(1, W.DT)


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_batch64_workload_properties(fx, orc, prec):
    """The 64 uneven MFIM instances at full size: after 2 + 1 steps every instance's phi
    satisfies the oracle's residual test for its P, and its last P is the oracle's TDGL update
    of the state before it."""
    inst = W.batch_instances(64)
    specs = [sp.copy(prec=prec) for sp, _ in inst]
    Ps = [P for _, P in inst]
    say(f"  64 instances, {sum(s.ncell for s in specs) / 1e6:.1f} M cells, prec={prec}")
    b = fx.Batch(specs, Ps)
    info = b.run(2, W.DT)
    assert all(i.status == fx.FX_OK and i.steps_done == 2 for i in info)
    Pa = [b.get(q, fx.FIELD_P) for q in range(64)]
    phia = [b.get(q, fx.FIELD_PHI) for q in range(64)]
    info = b.run(1, W.DT)
    worst_r = worst_p = 0.0
    for q, sp in enumerate(specs):
        P, phi = b.get(q, fx.FIELD_P), b.get(q, fx.FIELD_PHI)
        rn, fn = orc.residual_norms(sp, P, phi)
        worst_r = max(worst_r, rn / fn)
        P_o = orc.tdgl_step(sp, Pa[q], phia[q], W.DT)
        worst_p = max(worst_p, worst(sp, P, P_o))
        assert rn <= 1.5e-10 * fn, (q, rn / fn)
        assert worst(sp, P, P_o) <= 1e-13, q
        assert info[q].last_res_rel <= 1e-10
    say(f"  worst oracle residual {worst_r:.2e}, worst TDGL rel {worst_p:.2e}, "
        f"cycles/step {sum(i.total_cycles for i in info) / 64:.2f}")
