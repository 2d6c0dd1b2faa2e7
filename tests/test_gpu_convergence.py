"""The paper's convergence study (Methods, numerical validation; Table 2) on the GPU, at the
paper's sizes: the 32 nm MFISM cube with a Gaussian P bump, phi = 0 on both z-faces.

Tests 1 and 2 refine in time only (128^3 cells, 50 / 25 / 12.5 fs to 400 fs) with the
first- and second-order scheme; Test 3 refines in space only (64^3 / 128^3 / 256^3, 25 fs,
second-order scheme), comparing a finer field with a coarser one after averaging each 2x2x2
block of fine cells.  Rate = log2(E_c^m / E_m^f), E the RMS difference over the coarser grid.

The paper reports rates 1.00 / 1.01 (P / phi) for Test 1, 2.02 / 2.07 for Test 2 and
1.96 / 1.00 for Test 3.  The time rates are properties of the schemes and are checked to
+-0.1; the space rates depend on the interface discretisation (harmonic face permittivity
here) and are checked to be at least first order.  Before that, the GPU trajectories of this
workload match the oracle's element by element on a 32^3 cube.
"""
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W

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


def trajectory(fx, spec, dt, order):
    """The fields after 400 fs.  On 256^3 cells the residual of FP64 arithmetic stalls near
    2.5e-13 of |f|, so the finest grid is solved to 1e-11 (the space errors are ~1e-5)."""
    if spec.nx > 128:
        spec = spec.copy(tol_rel=1e-11)
    n = int(round(W.CONVERGENCE_T_END / dt))
    s = fx.Stack(spec.copy(time_order=order), W.gaussian_bump_P(spec))
    info = s.run_steps(n, dt)
    assert info.steps_done == n
    out = s.get(fx.FIELD_P), s.get(fx.FIELD_PHI), info.total_cycles / n
    s.close()
    return out


def rms(a):
    return float(np.sqrt(np.mean(a * a)))


def coarsen(a):
    n = a.shape[0] // 2
    return a.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))


@pytest.mark.parametrize("order", [1, 2])
def test_bump_trajectory_matches_oracle(fx, orc, order):
    spec = W.convergence_mfism(32)
    dt = W.CONVERGENCE_DT[0]
    P, phi, cyc = trajectory(fx, spec, dt, order)
    P_o, phi_o, _ = orc.run(spec, W.gaussian_bump_P(spec), 8, dt, tol=1e-13, order=order)
    rp, rf = rel(P, P_o), rel(phi, phi_o)
    say(f"  order {order}: cycles/step {cyc:.2f} relP {rp:.2e} relphi {rf:.2e}")
    assert rp <= 1e-10 and rf <= 1e-10


@pytest.mark.parametrize("order,paper", [(1, (1.00, 1.01)), (2, (2.02, 2.07))])
def test_table2_time_refinement(fx, order, paper):
    spec = W.convergence_mfism(128)
    res = [trajectory(fx, spec, dt, order) for dt in W.CONVERGENCE_DT]
    for f, name in ((0, "P"), (1, "phi")):
        e_cm = rms(res[1][f] - res[0][f])
        e_mf = rms(res[2][f] - res[1][f])
        rate = np.log2(e_cm / e_mf)
        say(f"  Test {order} {name}: E_c^m {e_cm:.3e} rate {rate:.3f} E_m^f {e_mf:.3e} "
            f"(paper rate {paper[f]:.2f}); cycles/step {res[0][2]:.2f} {res[1][2]:.2f} {res[2][2]:.2f}")
        assert rate == pytest.approx(order, abs=0.1)


def test_table2_space_refinement(fx):
    dt = W.CONVERGENCE_DT[1]
    res = [trajectory(fx, W.convergence_mfism(n), dt, 2) for n in (64, 128, 256)]
    for f, name, paper in ((0, "P", 1.96), (1, "phi", 1.00)):
        e_cm = rms(coarsen(res[1][f]) - res[0][f])
        e_mf = rms(coarsen(res[2][f]) - res[1][f])
        rate = np.log2(e_cm / e_mf)
        say(f"  Test 3 {name}: E_c^m {e_cm:.3e} rate {rate:.3f} E_m^f {e_mf:.3e} (paper rate {paper:.2f})")
        assert rate >= 0.9
