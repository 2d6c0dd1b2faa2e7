"""Parity at the benchmark's own size: the 256x256x128 MFISM stack (FE 48 / SiO2 8 / p-Si 64).

* Step 0 (the initial Poisson solve of the seeded P) against the oracle's Step 0 over every
  cell, FP64 and mixed precision, both solved to 1e-12 relative residual;
* the TDGL kernel over every ferroelectric cell, from the oracle's phi and the seeded P;
* in the benchmark's own launch configuration (tolerance 1e-10, extrapolated warm start, 5
  steps) a property that holds at any size: the oracle's own evaluation of the residual of
  the GPU's phi for the GPU's P meets the 1e-10 stopping rule after every step.
"""
import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W
from parity_check import worst

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def fx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_15668_amd import ferrox
    ferrox.lib()
    return ferrox


@pytest.fixture(scope="module")
def step0(orc):
    spec = W.mfism_large()
    P0 = W.random_P(spec, 2)
    print("  oracle Step 0 at 256x256x128 ...", flush=True)
    phi, info = orc.solve(spec, P0, tol=1e-12)
    return spec, P0, phi


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_fullsize_step0_parity(fx, step0, prec):
    spec, P0, phi_o = step0
    s = fx.Stack(spec.copy(prec=prec, tol_rel=1e-12), P0)
    e = worst(spec, s.get(fx.FIELD_PHI), phi_o)
    print(f"  prec {prec}: rel L2 phi {e:.2e}", flush=True)
    assert e <= 1e-10
    s.close()


def test_fullsize_tdgl_kernel(fx, orc, step0):
    spec, P0, phi_o = step0
    s = fx.Stack(spec, P0)
    s.set(fx.FIELD_PHI, phi_o)
    s.tdgl_step(W.DT)
    P_gpu = s.get(fx.FIELD_P)
    P_orc = orc.tdgl_step(spec, P0, phi_o, W.DT)
    assert worst(spec, P_gpu, P_orc) <= 1e-13
    f0, f1 = spec.fe_range()
    assert rel(P_gpu[f0:f1] - P0[f0:f1], P_orc[f0:f1] - P0[f0:f1]) <= 1e-11
    s.close()


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_fullsize_bench_configuration_residual(fx, orc, prec):
    spec = W.mfism_large(prec)                  # tol 1e-10, as timed by bench.py
    P0 = W.random_P(spec, 2)
    s = fx.Stack(spec, P0)
    for n in range(5):
        info = s.run_steps(1, W.DT)
        P, phi = s.get(fx.FIELD_P), s.get(fx.FIELD_PHI)
        rn, fn = orc.residual_norms(spec, P, phi)
        print(f"  step {n + 1}: {info.total_cycles} cycles, oracle |r|/|f| = {rn / fn:.3e}", flush=True)
        assert rn <= 1.05e-10 * fn
        f0, f1 = spec.fe_range()
        assert np.all(P[:f0] == 0) and np.all(P[f1:] == 0)
        assert np.all(np.isfinite(P)) and np.all(np.isfinite(phi))
    s.close()
