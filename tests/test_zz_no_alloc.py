"""poisson_solve_static, the entry point that allocates nothing (its workspace is the library's
static device array), against init_stack's Step 0 on the same inputs: the same kernels run, so
phi must agree bit for bit (and within the parity bound 1e-10 of the oracle comparisons).  Two
calls in a row, the second on a smaller stack, so the second runs in an array that still holds
the first call's contents."""
import sys

import numpy as np
import pytest

from paper_2210_15668_amd import workloads as W
from parity_check import check

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


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_static_solve_equals_init_stack_step0(fx, prec):
    import torch
    big = W.shrink_lateral(W.mfism_large(prec), 32, 32)
    small = W.layered(12, 16, 40, [(W.FE, 12, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0),
                                   (W.SC, 18, W.EPS_SI, 1e24)], v_top=-0.7, prec=prec)
    for q, spec in enumerate((big, small)):
        P0 = W.random_P(spec, 30 + q, amp=0.05)
        say(f"  call {q + 1}: {spec.nx}x{spec.ny}x{spec.nz} prec={prec}, static workspace")
        P = torch.from_numpy(P0).cuda()
        phi = torch.full((spec.nz, spec.ny, spec.nx), 123.0, dtype=torch.float64, device="cuda")
        info = fx.poisson_solve_static(spec, P, phi)
        torch.cuda.synchronize()
        ref = fx.Stack(spec, P0)
        phi_ref = ref.get(fx.FIELD_PHI)
        got = phi.cpu().numpy()
        say(f"    {info.cycles} V-cycles, |r| {info.res_norm:.3e} |f| {info.rhs_norm:.3e}; "
            f"max |diff| vs init_stack {np.abs(got - phi_ref).max():.3e}")
        check(spec, got, phi_ref, 1e-10, "phi vs init_stack")
        assert np.array_equal(got, phi_ref)
        assert info.status == fx.FX_OK and info.res_norm <= spec.tol_rel * info.rhs_norm
        assert np.array_equal(P.cpu().numpy(), ref.get(fx.FIELD_P))
        ref.close()


def test_static_solve_rejects_a_stack_beyond_the_array(fx):
    import torch
    spec = W.mfism_large()                     # needs about 0.56 GB of workspace
    P = torch.zeros((spec.nz, spec.ny, spec.nx), dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(P)
    with pytest.raises(fx.FerroxError) as e:
        fx.poisson_solve_static(spec, P, phi)
    assert e.value.status == fx.FX_ENOMEM
