"""Pins of the CPU float64 U-Net reference (oracle/unet_ref.py) against facts that do not
come from the reference itself: central finite differences of the loss, adjoint
identities of each operator, closed forms of a convolution, the network's equivariance
under lateral shifts, and the series-capacitor profile against the independently written
Poisson oracle."""
import numpy as np
import pytest

from oracle import unet_ref as U
from paper_2210_15668_amd import workloads as W


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_parameter_count_and_layout():
    n = U.num_params()
    assert n == sum(27 * ci * co + co for _, ci, co in U.LAYERS) + 17
    theta = np.arange(n, dtype=np.float64)
    p = U.unpack(theta)
    W0, b0 = p["e0a"]
    assert W0.shape == (27, 16, 16) and W0[0, 0, 0] == 0 and W0[0, 0, 1] == 1 and W0[0, 1, 0] == 16
    assert b0[0] == 27 * 16 * 16
    w, b = p["head"]
    assert w.shape == (16,) and b[0] == n - 1


def test_conv_identity_tap():
    x = rnd((4, 4, 4, 5), 1)
    Wt = np.zeros((27, 5, 5))
    Wt[13] = np.eye(5)                      # tap (0, 0, 0)
    assert np.array_equal(U.conv3(x, Wt, np.zeros(5)), x)


def test_conv_of_a_constant_field_closed_form():
    """Interior planes see all 27 taps; the bottom plane only taps with dz >= 0."""
    D, C = 6, 3
    x = np.zeros((D, 4, 4, C))
    x[..., 1] = 2.5
    Wt = rnd((27, 2, C), 2)
    b = rnd(2, 3)
    y = U.conv3(x, Wt, b)
    full = b + 2.5 * Wt[:, :, 1].sum(axis=0)
    bottom = b + 2.5 * Wt[9:, :, 1].sum(axis=0)          # taps with dz in {0, 1}
    top = b + 2.5 * Wt[:18, :, 1].sum(axis=0)            # dz in {-1, 0}
    assert np.allclose(y[2], full, rtol=1e-13, atol=1e-13)
    assert np.allclose(y[0], bottom, rtol=1e-13, atol=1e-13)
    assert np.allclose(y[D - 1], top, rtol=1e-13, atol=1e-13)


def test_conv_tap_reads_the_stated_neighbour():
    """A single nonzero weight at tap (dz, dy, dx) = (1, -1, 1) copies x[z+1, y-1, x+1]."""
    x = rnd((4, 5, 6, 1), 4)
    Wt = np.zeros((27, 1, 1))
    Wt[(1 + 1) * 9 + (-1 + 1) * 3 + (1 + 1)] = 1.0
    y = U.conv3(x, Wt, np.zeros(1))
    for z in range(3):
        for yy in range(5):
            for xx in range(6):
                assert y[z, yy, xx, 0] == x[z + 1, (yy - 1) % 5, (xx + 1) % 6, 0]
    assert np.all(y[3] == 0.0)


def test_adjoint_identities():
    x = rnd((4, 6, 8, 3), 5)
    g = rnd((4, 6, 8, 2), 6)
    Wt = rnd((27, 2, 3), 7)
    y = U.conv3(x, Wt, np.zeros(2))
    gx, gW, gb = U.conv3_backward(x, Wt, g)
    lhs = np.sum(y * g)
    assert np.isclose(lhs, np.sum(x * gx), rtol=1e-12)
    assert np.isclose(lhs, np.sum(Wt * gW), rtol=1e-12)        # y is linear in W
    assert np.allclose(gb, g.sum(axis=(0, 1, 2)))
    a = rnd((2, 3, 4, 2), 8)
    bb = rnd((4, 6, 8, 2), 9)
    assert np.isclose(np.sum(U.up(a) * bb), np.sum(a * U.up_backward(bb)), rtol=1e-12)
    c = rnd((4, 6, 8, 2), 10)
    d = rnd((2, 3, 4, 2), 11)
    assert np.isclose(np.sum(U.pool(c) * d), np.sum(c * U.pool_backward(d)), rtol=1e-12)
    assert np.allclose(U.pool(U.up(a)), a, rtol=1e-15)


def test_network_is_equivariant_under_lateral_shifts_by_four():
    theta = U.init_params(3)
    x = rnd((8, 8, 12, 16), 12)
    out = U.forward(theta, x)
    xs = np.roll(x, shift=(4, 8), axis=(1, 2))
    assert np.allclose(U.forward(theta, xs), np.roll(out, shift=(4, 8), axis=(1, 2)), rtol=1e-12, atol=1e-12)
    # not along z: the z-ends see zeros
    xz = np.roll(x, shift=4, axis=0)
    assert not np.allclose(U.forward(theta, xz), np.roll(out, shift=4, axis=0), atol=1e-6)


def test_gradient_matches_central_differences():
    theta = U.init_params(5)
    theta += 0.05 * rnd(theta.shape, 13)        # nonzero biases too
    x = rnd((8, 8, 8, 16), 14)
    x[..., 3:] = 0.0
    target = rnd((8, 8, 8), 15)
    L, g = U.gradient(theta, x, target)
    assert np.isclose(L, U.loss(theta, x, target), rtol=1e-14)
    rng = np.random.default_rng(16)
    offs = [0]
    for _, ci, co in U.LAYERS:
        offs.append(offs[-1] + 27 * ci * co + co)
    idx = []
    for q in range(len(U.LAYERS)):
        idx += list(rng.integers(offs[q], offs[q + 1], 3))     # weights and maybe biases
        idx.append(offs[q + 1] - 1)                             # the layer's last bias
    idx += [offs[-1] + 3, U.num_params() - 1]                   # head weight, head bias
    h = 1e-6
    worst = 0.0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (U.loss(tp, x, target) - U.loss(tm, x, target)) / (2 * h)
        err = abs(fd - g[i]) / max(abs(g[i]), 1e-8)
        worst = max(worst, err)
        assert err <= 1e-5, (i, fd, g[i])
    assert worst <= 1e-5


def test_phi_lin_is_the_p0_solution_of_the_linear_stack(orc):
    """With P = 0 and no semiconductor the discrete Poisson solution is the series
    capacitor at the cell centres: the Poisson oracle (its own code) must agree."""
    spec = W.layered(4, 4, 26, [(W.FE, 12, W.EPS_FE, 0.0), (W.DE, 4, W.EPS_SIO2, 0.0),
                                (W.DE, 5, W.EPS_AL2O3, 0.0)], v_top=1.3, v_bottom=-0.2)
    phi, _ = orc.solve(spec, np.zeros((spec.nz, spec.ny, spec.nx)), tol=1e-14)
    kb, kt = spec.device_range()
    lin = U.phi_lin(spec, 1.3)
    assert np.allclose(phi[kb:kt, 1, 2], lin, rtol=0, atol=1e-12)


def test_pack_and_unpack_round_trip():
    spec = W.shrink_lateral(W.mfism_medium(), 8, 8)
    rng = np.random.default_rng(17)
    P = W.random_P(spec, 18, amp=0.1)
    phi = rng.standard_normal((spec.nz, spec.ny, spec.nx))
    x = U.pack_input(spec, P, -1.5)
    kb, kt = spec.device_range()
    f0, f1 = spec.fe_range()
    assert x.shape == (kt - kb, 8, 8, 16)
    assert np.array_equal(x[f0 - kb:f1 - kb, ..., 0], P[f0:f1] / U.P_SCALE)
    assert np.all(x[..., 2] == -1.5 / U.V_SCALE) and np.all(x[..., 3:] == 0)
    sc = spec.plane_mat[kb:kt] == W.SC
    assert np.all(x[sc, ..., 1] == -1.0) and np.all(x[~sc, ..., 1] == 0.0)
    t = U.pack_target(spec, phi, -1.5)
    assert np.allclose(U.unpack_prediction(spec, t, -1.5), phi[kb:kt], rtol=0, atol=1e-14)



def test_rounding_hooks_default_to_the_float64_network():
    theta = U.init_params(21)
    x = rnd((8, 8, 8, 16), 22)
    t = rnd((8, 8, 8), 23)
    L0, g0 = U.gradient(theta, x, t)
    L1, g1 = U.gradient(theta, x, t, rnd=lambda v: v, grnd=lambda v: v)
    assert L0 == L1 and np.array_equal(g0, g1)
    # a rounding hook is applied where stated: rounding activations to integers changes the output
    assert not np.allclose(U.forward(theta, x, rnd=np.round), U.forward(theta, x))


def test_dyadic_inputs_are_exact_in_fp32_in_any_order():
    """On the dyadic test inputs (tests/unet_dyadic.py) a float32 evaluation that sums in
    another order reproduces the float64 reference with BF16 rounding hooks bit for bit, in
    every activation and every back-propagated signal: the premise of the GPU gradient test's
    tight bound.  With random He-normal weights the same two evaluations part (near-tie
    roundings flip and the flips cascade), which is why that test needs these inputs."""
    import unet_dyadic as D
    shape = (8, 8, 16)
    for seed in (1, 2):
        th, x, t = D.params(seed), D.inputs(seed + 1, shape), D.target(seed + 2, shape)
        L, g, sig = U.gradient(th, x, t, rnd=D.bf16, grnd=D.bf16, keep=True)
        out_r, a_r = U.forward(th, x, keep=True, rnd=D.bf16)
        out_e, a_e, sig_e = D.emulate_fp32(th, x, t)
        assert np.array_equal(out_r, out_e.astype(np.float64))
        for k in a_r:
            if not k.endswith(".in"):
                assert np.array_equal(a_r[k], a_e[k].astype(np.float64)), k
                assert 0.1 < np.mean(a_r[k] > 0) < 0.9, k          # ReLUs neither dead nor linear
        for k in sig:
            assert np.array_equal(sig[k], sig_e[k].astype(np.float64)), k
        for name, _, _ in U.LAYERS:
            assert np.linalg.norm(U.unpack(g)[name][0]) > 1e-3, name   # every layer gets a gradient
    # random weights: the same comparison is not exact (the reason for the dyadic inputs)
    th = D.params(3)
    th[:] = U.init_params(3)
    x = D.inputs(4, shape)
    x[..., :3] = np.random.default_rng(5).uniform(-1, 1, shape + (3,))
    x = D.bf16(x)
    out_r = U.forward(th, x, rnd=D.bf16)
    out_e, _, _ = D.emulate_fp32(th, x, D.target(6, shape))
    assert not np.array_equal(out_r, out_e.astype(np.float64))
