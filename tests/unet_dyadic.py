"""Network inputs on which BF16-operand / FP32-accumulation arithmetic is exact.

Every weight is 0 or +-2^-k with k from a small range (a few nonzero taps and channels per
output channel), every bias a multiple of 1/8, every input value 0, +-1/2 or +-1, every
target a multiple of 2^-7, and the cell count a power of two (so 2/n is exact).  Then each
pre-activation, pooled sum, back-propagated signal and head output is a sum of products on a
coarse binary grid that fits FP32's 24-bit significand, whatever the summation order: an FP32
evaluation with BF16 rounding at the stored activations and signals reproduces the float64
reference with the same rounding hooks bit for bit (checked on the CPU by `emulate_fp32`,
which sums the taps in reverse order).  Only the final reductions over voxels (weight and bias
gradients, the loss) may differ, by FP32 rounding.  The GPU kernels round at those same
points, so on these inputs a rounding point placed differently, a wrong tap, channel or
layout, or a scaled gradient shows as a gross difference instead of hiding inside the
accumulated BF16 noise of random data.
"""
import numpy as np

from oracle import unet_ref as U


def bf16(x):
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def params(seed, nnz=16, kmin=2, kmax=3):
    rng = np.random.default_rng(seed)
    th = np.zeros(U.num_params())
    p = U.unpack(th)
    for name, ci, co in U.LAYERS:
        W, b = p[name]
        cin_used = 3 if name == "e0a" else ci
        for o in range(co):
            for _ in range(nnz):
                t, c = rng.integers(27), rng.integers(cin_used)
                W[t, o, c] = rng.choice([-1.0, 1.0]) * 2.0 ** -rng.integers(kmin, kmax + 1)
        b[:] = rng.integers(-2, 3, co) * 0.125
    w, b = p["head"]
    w[:] = rng.choice([-1.0, 1.0], 16) * 2.0 ** -rng.integers(1, 4, 16)
    b[0] = 0.0625
    return th


def inputs(seed, shape):
    rng = np.random.default_rng(seed)
    x = np.zeros(tuple(shape) + (16,))
    x[..., :3] = rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], tuple(shape) + (3,))
    return x


def target(seed, shape):
    return np.random.default_rng(seed).integers(-128, 129, shape) * 2.0 ** -7


def _conv32(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[1],), np.float32) + b.astype(np.float32)
    for t, dz, dy, dx in list(U.taps())[::-1]:
        y += U.shift(x, dz, dy, dx).astype(np.float32) @ W[t].T.astype(np.float32)
    return y


def emulate_fp32(theta, x, tgt):
    """The network in float32 with BF16 rounding of activations and signals, taps summed in
    reverse order: returns (output, activations, signals entering each backward conv)."""
    f = np.float32
    p = U.unpack(theta)
    a = {}

    def layer(name, inp):
        W, b = p[name]
        out = bf16(np.maximum(_conv32(inp, W, b), 0)).astype(np.float32)
        a[name] = out
        a[name + ".in"] = inp
        return out

    def pool32(v):
        D, H, Wd, C = v.shape
        s = v.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).astype(np.float32).sum(axis=(1, 3, 5))
        return bf16(s * f(0.125)).astype(np.float32)

    s0 = layer("e0b", layer("e0a", x.astype(np.float32)))
    s1 = layer("e1b", layer("e1a", pool32(s0)))
    bt = layer("b2b", layer("b2a", pool32(s1)))
    u1 = layer("d1b", layer("d1a", np.concatenate([U.up(bt), s1], 3)))
    u0 = layer("d0b", layer("d0a", np.concatenate([U.up(u1), s0], 3)))
    w, b = p["head"]
    out = (u0 @ w.astype(np.float32) + f(b[0])).astype(np.float32)
    d_out = f(2.0 / out.size) * (out - tgt.astype(np.float32))
    sig = {}

    def back(name, dy):
        W, _ = p[name]
        dz = bf16(dy * (a[name] > 0)).astype(np.float32)
        sig[name] = dz
        gx = np.zeros(a[name + ".in"].shape, np.float32)
        for t, dzz, dyy, dxx in list(U.taps())[::-1]:
            gx += U.shift_adjoint(dz @ W[t].astype(np.float32), dzz, dyy, dxx)
        return gx

    d = back("d0a", back("d0b", d_out[..., None] * w.astype(np.float32)))
    c = a["d1b"].shape[3]
    d_u1, d_s0 = U.up_backward(d[..., :c]), d[..., c:].copy()
    d = back("d1a", back("d1b", d_u1))
    c = a["b2b"].shape[3]
    d_bt, d_s1 = U.up_backward(d[..., :c]), d[..., c:].copy()
    d = back("b2a", back("b2b", d_bt))
    d_s1 += U.pool_backward(d).astype(np.float32)
    d = back("e1a", back("e1b", d_s1))
    d_s0 += U.pool_backward(d).astype(np.float32)
    back("e0a", back("e0b", d_s0))
    return out, a, sig
