"""Solver choices that must not change results.  The fused launches below the finest level
(the zero-start red/black pair; on small levels the prolongation formed inside the first
red half-sweep; on small red/black levels the blocked smoothing, where the pre-smoothing
sweeps with the restriction and the prolongation with the post-smoothing sweeps are one
launch each over LDS tiles) reproduce the separate launches bit for bit (FERROX_FUSE=0
keeps every half-sweep and transfer a launch of its own), for single stacks in both
precisions and for a batch, and the fused stack meets the oracle's 1e-10 parity bar.  Light cycles and
either coarsening stop (8 or 64 bottom cells) change the cycles, not the root."""
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_15668_amd import ferrox
    ferrox.lib()
    return ferrox


def run_stack(fx, monkeypatch, fuse, spec, P0, n, modes=None):
    monkeypatch.setenv("FERROX_FUSE", fuse)
    s = fx.Stack(spec, P0)
    if modes is not None:
        modes.extend(s.level_modes())
    info = s.run_steps(n, W.DT)
    out = s.get(fx.FIELD_P), s.get(fx.FIELD_PHI), info.total_cycles
    s.close()
    return out


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_fused_equals_separate_launches_on_a_stack(fx, orc, monkeypatch, prec):
    # 64 x 64 MFISM: levels 1.. are red/black and under 2^18 cells, so both fusions run
    spec = W.shrink_lateral(W.mfism_large(prec), 64, 64).copy(tol_rel=1e-12)
    P0 = W.random_P(spec, 90, amp=0.05)
    n = 6
    say(f"  prec {prec}: fused ...")
    mf, ms = [], []
    Pf, phif, cf = run_stack(fx, monkeypatch, "1", spec, P0, n, mf)
    say(f"  prec {prec}: separate ...")
    Ps, phis, cs = run_stack(fx, monkeypatch, "0", spec, P0, n, ms)
    say(f"  V-cycles fused {cf} separate {cs}; level modes fused {mf} separate {ms}")
    assert fx.LEVEL_BLOCKED in mf and fx.LEVEL_BLOCKED not in ms
    assert cf == cs
    assert np.array_equal(Pf, Ps) and np.array_equal(phif, phis)
    if prec == W.PREC_FP64:
        P_o, phi_o, _ = orc.run(spec, P0, n, W.DT, tol=1e-12)
        rp, rf = rel(Pf, P_o), rel(phif, phi_o)
        say(f"  vs oracle: relP {rp:.2e} relphi {rf:.2e}")
        assert rp <= 1e-10 and rf <= 1e-10


def test_fused_equals_separate_launches_in_a_batch(fx, monkeypatch):
    specs = [W.layered(32, 32, 32, [(W.FE, 16, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)], v_top=0.5,
                       tol_rel=1e-12),
             W.layered(48, 32, 48, [(W.FE, 24, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0),
                                    (W.SC, 12, W.EPS_SI, 1e24)], v_top=-0.8, tol_rel=1e-12, time_order=2)]
    Ps = [W.random_P(sp, 91 + q, amp=0.05) for q, sp in enumerate(specs)]
    out = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("FERROX_FUSE", fuse)
        b = fx.Batch(specs, Ps)
        info = b.run(5, W.DT)
        assert all(i.status == fx.FX_OK and i.steps_done == 5 for i in info)
        out[fuse] = [(b.get(q, fx.FIELD_P), b.get(q, fx.FIELD_PHI)) for q in range(len(specs))]
        b.close()
    for q in range(len(specs)):
        assert np.array_equal(out["1"][q][0], out["0"][q][0]) and np.array_equal(out["1"][q][1], out["0"][q][1]), q


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
@pytest.mark.parametrize("nu", ["1", "2"])
def test_blocked_smoothing_equals_launches(fx, monkeypatch, prec, nu):
    """The blocked smoothing (FERROX_TB=1, the default) against the same levels launched
    half-sweep by half-sweep with every other fusion kept (FERROX_TB=0): the same bits, with
    one or two sweeps before and after the coarse correction on the levels below the finest
    (nu), light cycles included.  The 128 x 128 x 64 MFIM of the ramp (a 48-plane device
    slab) runs its levels 64 x 64 x 24 and 32 x 32 x 12 blocked."""
    monkeypatch.setenv("FERROX_NU1C", nu)
    monkeypatch.setenv("FERROX_NU2C", nu)
    spec = W.mfim_ramp().copy(tol_rel=1e-12, prec=prec, v_top=1.0)
    P0 = W.random_P(spec, 95, amp=0.05)
    n = 6
    out = {}
    for tb in ("1", "0"):
        monkeypatch.setenv("FERROX_TB", tb)
        s = fx.Stack(spec, P0)
        modes = s.level_modes()
        info = s.run_steps(n, W.DT)
        out[tb] = (s.get(fx.FIELD_P), s.get(fx.FIELD_PHI), info.total_cycles, modes)
        s.close()
    say(f"  prec {prec} nu {nu}: level modes {out['1'][3]} / {out['0'][3]}, V-cycles {out['1'][2]} / {out['0'][2]}")
    assert out["1"][3].count(fx.LEVEL_BLOCKED) >= 2 and fx.LEVEL_BLOCKED not in out["0"][3]
    assert out["1"][2] == out["0"][2]
    assert np.array_equal(out["1"][0], out["0"][0]) and np.array_equal(out["1"][1], out["0"][1])


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_blocked_smoothing_equals_launches_in_a_batch(fx, monkeypatch, prec):
    """A batch of uneven instances whose levels below the finest all qualify (lateral sizes
    multiples of 16, at most 30 planes there), some with semiconductor planes: blocked
    smoothing against FERROX_TB=0, every instance bit for bit."""
    specs = []
    for q, (nx, ny, nz) in enumerate([(64, 64, 48), (96, 64, 48), (64, 96, 40), (128, 64, 48)]):
        layers = [(W.FE, 16 + 4 * q, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)]
        if q % 2:
            layers.append((W.SC, 16, W.EPS_SI, 1e24))
        specs.append(W.layered(nx, ny, nz, layers, v_top=1.0 - 0.5 * q, tol_rel=1e-12, prec=prec,
                               **({"ni": 1.0e16, "T": 300.0} if q % 2 else {})))
    Ps = [W.random_P(sp, 96 + q, amp=0.05) for q, sp in enumerate(specs)]
    out, modes = {}, {}
    for tb in ("1", "0"):
        monkeypatch.setenv("FERROX_TB", tb)
        b = fx.Batch(specs, Ps)
        modes[tb] = b.level_modes()
        info = b.run(5, W.DT)
        assert all(i.status == fx.FX_OK and i.steps_done == 5 for i in info)
        out[tb] = [(b.get(q, fx.FIELD_P), b.get(q, fx.FIELD_PHI)) for q in range(len(specs))]
        b.close()
    say(f"  prec {prec}: batch level modes {modes['1']} / {modes['0']}")
    assert fx.LEVEL_BLOCKED in modes["1"] and fx.LEVEL_BLOCKED not in modes["0"]
    for q in range(len(specs)):
        assert np.array_equal(out["1"][q][0], out["0"][q][0]) and np.array_equal(out["1"][q][1], out["0"][q][1]), q


# (lateral x, lateral y, layers gate-first, the level-1 shape that is to run blocked)
TB_EDGES = [
    # 30 planes on level 1: the most a box holds (its FP64 LDS is 63 KB of 64); the finest
    # level's odd 59th plane is left unpaired
    (32, 32, [(W.FE, 24, W.EPS_FE, 0.0), (W.DE, 5, W.EPS_SIO2, 0.0), (W.SC, 30, W.EPS_SI, 1e24)], (16, 16, 30)),
    # an odd plane count on the blocked level itself (29 into 15: the top coarse plane
    # has one child), semiconductor planes below
    (32, 32, [(W.FE, 20, W.EPS_FE, 0.0), (W.DE, 6, W.EPS_SIO2, 0.0), (W.SC, 32, W.EPS_SI, 1e24)], (16, 16, 29)),
    # extents that are multiples of the 8-cell tile but not of the 16-cell box: 3 x 5 tiles
    (48, 80, [(W.FE, 32, W.EPS_FE, 0.0), (W.DE, 8, W.EPS_SIO2, 0.0)], (24, 40, 20)),
]


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
@pytest.mark.parametrize("case", range(len(TB_EDGES)))
def test_blocked_smoothing_at_its_geometry_limits(fx, orc, monkeypatch, prec, case):
    """Blocked smoothing where its geometry is tightest (box planes at the LDS limit, an odd
    plane count with an unpaired top plane, tiles that do not fill a whole box): the blocked
    level runs blocked, the result is bitwise that of the half-sweep launches (FERROX_TB=0),
    and in FP64 it meets the oracle's trajectory to 1e-10."""
    nx, ny, layers, shape = TB_EDGES[case]
    nzd = sum(l[1] for l in layers)
    sc = any(l[0] == W.SC for l in layers)
    spec = W.layered(nx, ny, nzd + 4, layers, v_top=0.7, tol_rel=1e-12, prec=prec,
                     **({"ni": 1.0e16, "T": 300.0} if sc else {}))
    P0 = W.random_P(spec, 97 + case, amp=0.05)
    n = 5
    out = {}
    for tb in ("1", "0"):
        monkeypatch.setenv("FERROX_TB", tb)
        s = fx.Stack(spec, P0)
        shapes, modes = s.levels(), s.level_modes()
        info = s.run_steps(n, W.DT)
        assert info.steps_done == n
        out[tb] = (s.get(fx.FIELD_P), s.get(fx.FIELD_PHI), info.total_cycles, shapes, modes)
        s.close()
    shapes, modes = out["1"][3], out["1"][4]
    say(f"  prec {prec} case {case}: levels {shapes}, modes {modes} / {out['0'][4]}, "
        f"V-cycles {out['1'][2]} / {out['0'][2]}")
    assert shapes[1] == shape and modes[1] == fx.LEVEL_BLOCKED and fx.LEVEL_BLOCKED not in out["0"][4]
    assert out["1"][2] == out["0"][2]
    assert np.array_equal(out["1"][0], out["0"][0]) and np.array_equal(out["1"][1], out["0"][1])
    if prec == W.PREC_FP64:
        P_o, phi_o, _ = orc.run(spec, P0, n, W.DT, tol=1e-12)
        rp, rf = rel(out["1"][0], P_o), rel(out["1"][1], phi_o)
        say(f"  vs oracle: relP {rp:.2e} relphi {rf:.2e}")
        assert rp <= 1e-10 and rf <= 1e-10


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_light_cycles_reach_the_oracle_root(fx, orc, monkeypatch, prec):
    """Light cycles (one sweep fewer per level after a cycle that left the residual near the
    tolerance) change the iterates, not the root: with and without them the run meets the
    oracle's trajectory to 1e-10."""
    spec = W.shrink_lateral(W.mfism_large(prec), 32, 32).copy(tol_rel=1e-13)
    P0 = W.random_P(spec, 92, amp=0.05)
    n = 12
    P_o, phi_o, _ = orc.run(spec, P0, n, W.DT, tol=1e-13)
    for light in ("1", "0"):
        monkeypatch.setenv("FERROX_LIGHT", light)
        s = fx.Stack(spec, P0)
        info = s.run_steps(n, W.DT)
        rp, rf = rel(s.get(fx.FIELD_P), P_o), rel(s.get(fx.FIELD_PHI), phi_o)
        say(f"  prec {prec} light {light}: cycles {info.total_cycles} relP {rp:.2e} relphi {rf:.2e}")
        assert info.steps_done == n and rp <= 1e-10 and rf <= 1e-10
        s.close()


@pytest.mark.parametrize("cells", ["8", "64"])
def test_bottom_size_reaches_the_oracle_root(fx, orc, monkeypatch, cells):
    """The size at which coarsening stops (FERROX_BOTTOM_CELLS; 64 lets the one-wave conjugate
    gradients take a 4x4x2 bottom) changes the cycles, not the root."""
    monkeypatch.setenv("FERROX_BOTTOM_CELLS", cells)
    spec = W.shrink_lateral(W.mfism_large(), 32, 32).copy(tol_rel=1e-13)
    P0 = W.random_P(spec, 93, amp=0.05)
    n = 6
    s = fx.Stack(spec, P0)
    info = s.run_steps(n, W.DT)
    levels = fx.lib().stack_num_levels(s._h)
    P_o, phi_o, _ = orc.run(spec, P0, n, W.DT, tol=1e-13)
    rp, rf = rel(s.get(fx.FIELD_P), P_o), rel(s.get(fx.FIELD_PHI), phi_o)
    say(f"  bottom <= {cells} cells: {levels} levels, cycles {info.total_cycles} relP {rp:.2e} relphi {rf:.2e}")
    assert info.steps_done == n and rp <= 1e-10 and rf <= 1e-10
    s.close()


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_coarse_column_prolongation_is_bitwise(fx, monkeypatch, prec):
    """The prolongation by coarse columns (a thread per coarse column marching in z, reusing
    each plane's bilinear values) forms every correction with the operands and order of the
    per-fine-cell kernel (FERROX_PROLONG_CC=0): same bits, on a stack whose first two levels
    take it (160 x 160 lateral, level 1 above the fused small-level limit) and in a batch."""
    spec = W.shrink_lateral(W.mfism_large(prec), 160, 160).copy(tol_rel=1e-12)
    P0 = W.random_P(spec, 94, amp=0.05)
    specs = [W.layered(96, 64, 48, [(W.FE, 30, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0)], v_top=0.5,
                       tol_rel=1e-12, prec=prec),
             W.layered(48, 32, 47, [(W.FE, 24, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0),
                                    (W.SC, 11, W.EPS_SI, 1e24)], v_top=-0.8, tol_rel=1e-12, time_order=2, prec=prec)]
    Ps = [W.random_P(sp, 95 + q, amp=0.05) for q, sp in enumerate(specs)]
    out = {}
    for cc in ("1", "0"):
        monkeypatch.setenv("FERROX_PROLONG_CC", cc)
        s = fx.Stack(spec, P0)
        info = s.run_steps(4, W.DT)
        b = fx.Batch(specs, Ps)
        bi = b.run(4, W.DT)
        assert all(i.status == fx.FX_OK for i in bi)
        out[cc] = (s.get(fx.FIELD_P), s.get(fx.FIELD_PHI), info.total_cycles,
                   [(b.get(q, fx.FIELD_P), b.get(q, fx.FIELD_PHI)) for q in range(len(specs))])
        say(f"  prolong by coarse columns {cc}: {info.total_cycles} V-cycles")
        s.close()
        b.close()
    a, c = out["1"], out["0"]
    assert a[2] == c[2] and np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    for q in range(len(specs)):
        assert np.array_equal(a[3][q][0], c[3][q][0]) and np.array_equal(a[3][q][1], c[3][q][1]), q
