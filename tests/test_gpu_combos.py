"""Feature combinations on the GPU: the predictor-corrector with Fermi-Dirac carriers and
mixed precision, recorded Q-V runs in graph replay, warm-start orders under the second-order
scheme, and degenerate calls (no steps, a batch of one).  Every field is compared with the
oracle's scheme of the same options to 1e-10, and Q / V_fe to 1e-8 (see test_gpu_qv)."""
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W
from parity_check import worst

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


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


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_predictor_corrector_with_fermi_dirac_recorded_in_a_graph_batch(fx, orc, prec):
    base = W.mfism_fig4(16, prec).copy(tol_rel=1e-13)
    specs = [base.copy(time_order=2, v_top=0.8),
             base.copy(time_order=1, v_top=-0.6),
             W.shrink_lateral(W.mfism_large(prec), 16, 16).copy(tol_rel=1e-13, time_order=2,
                                                                carriers=W.CARRIERS_FD)]
    Ps = [W.random_P(sp, 80 + q, amp=0.1) for q, sp in enumerate(specs)]
    n = 6
    vs = [sp.v_top + 0.2 * np.arange(1, n + 1) / n for sp in specs]
    rec = {}
    for mode in (fx.LAUNCH_GRAPH, fx.LAUNCH_STREAM):
        b = fx.Batch(specs, Ps)
        b.set_launch(mode)
        info, Q, V = b.run_qv(n, W.DT_TABLE1, vs)
        assert all(i.status == fx.FX_OK and i.steps_done == n for i in info)
        rec[mode] = (Q, V, [b.get(q, fx.FIELD_PHI) for q in range(len(specs))])
        if mode == fx.LAUNCH_GRAPH:
            for q, sp in enumerate(specs):
                P_o, phi_o, _ = orc.run(sp, Ps[q], n, W.DT_TABLE1, v_sched=vs[q], tol=1e-13, order=sp.time_order)
                rp, rf = worst(sp, b.get(q, fx.FIELD_P), P_o), worst(sp, b.get(q, fx.FIELD_PHI), phi_o)
                Qo, Vo = orc.qv(sp.copy(v_top=vs[q][-1]), P_o, phi_o)
                say(f"  inst {q} order {sp.time_order} carriers {sp.carriers}: relP {rp:.2e} relphi {rf:.2e} "
                    f"Q {Q[q][-1]:.6e} ({Qo:.6e})")
                assert rp <= 1e-10 and rf <= 1e-10, q
                assert abs(Q[q][-1] - Qo) <= 1e-8 * abs(Qo) and abs(V[q][-1] - Vo) <= 1e-8 * abs(Vo), q
        b.close()
    g, st = rec[fx.LAUNCH_GRAPH], rec[fx.LAUNCH_STREAM]
    for q in range(len(specs)):
        assert np.array_equal(g[0][q], st[0][q]) and np.array_equal(g[1][q], st[1][q])
        assert np.array_equal(g[2][q], st[2][q])


@pytest.mark.parametrize("warm", [0, 1, 3])
def test_predictor_corrector_under_every_warm_start(fx, orc, warm):
    spec = W.mfim_small().copy(tol_rel=1e-13, time_order=2, warm_start=warm)
    P0 = W.random_P(spec, 81, amp=0.1)
    s = fx.Stack(spec, P0)
    info = s.run_steps(8, W.DT)
    P_o, phi_o, _ = orc.run(spec, P0, 8, W.DT, tol=1e-13, order=2)
    say(f"  warm {warm}: cycles/step {info.total_cycles / 8:.2f}")
    assert worst(spec, s.get(fx.FIELD_P), P_o) <= 1e-10 and worst(spec, s.get(fx.FIELD_PHI), phi_o) <= 1e-10


def test_single_stack_graph_replay_is_bitwise_for_both_schemes(fx):
    for order in (1, 2):
        spec = W.shrink_lateral(W.mfism_large(), 16, 16).copy(tol_rel=1e-12, time_order=order)
        P0 = W.random_P(spec, 82, amp=0.05)
        out = []
        for mode in (fx.LAUNCH_STREAM, fx.LAUNCH_GRAPH):
            s = fx.Stack(spec, P0)
            s.set_launch(mode)
            s.run_steps(7, W.DT)
            out.append((s.get(fx.FIELD_P), s.get(fx.FIELD_PHI)))
            s.close()
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1]), order


def test_degenerate_calls(fx, orc):
    """No steps leave everything as it was; a batch of one equals the stack."""
    spec = W.mfim_small().copy(tol_rel=1e-12, time_order=2)
    P0 = W.random_P(spec, 83, amp=0.05)
    s = fx.Stack(spec, P0)
    phi0 = s.get(fx.FIELD_PHI)
    info, Q, V = s.run_steps_qv(0, W.DT)
    assert info.steps_done == 0 and Q.size == 0
    assert np.array_equal(s.get(fx.FIELD_PHI), phi0)
    s.run_steps(3, W.DT)
    b = fx.Batch([spec], [P0])
    b.run(3, W.DT)
    assert np.array_equal(b.get(0, fx.FIELD_PHI), s.get(fx.FIELD_PHI))
    assert np.array_equal(b.get(0, fx.FIELD_P), s.get(fx.FIELD_P))
