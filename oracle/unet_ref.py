"""CPU float64 reference of the learned warm start's network -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use this module;
the product path (the HIP library) neither imports nor calls it.

The network is the learned warm start of the Poisson solve: a small 3D convolutional
U-Net maps per-cell inputs (the polarisation P_z, the doping, and the gate voltage as a
broadcast channel) on the device slab to the deviation of phi from the P = 0
series-capacitor profile phi_lin(V).  The architecture is fixed: three levels with 16, 32
and 64 channels, two 3x3x3 convolutions (each followed by ReLU) per level on the way down
and on the way up, 2x2x2 average pooling, nearest-neighbour 2x upsampling, skip
connections by channel concatenation, and a 1x1x1 linear head.

Conventions (shared with the HIP library by specification, not by code):
  * tensors are (D, H, W, C) = (z, y, x, channel) over the device planes;
  * convolutions wrap periodically in x and y (the device is periodic there) and see
    zeros beyond the two z-ends;
  * a 3x3x3 kernel tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), d in {-1, 0, 1}, reads the input
    at (z+dz, y+dy, x+dx); weights are stored per layer as W[t][cout][cin], then b[cout];
    the head stores w[16], then b;
  * the flat parameter vector lists the layers in LAYERS order, then the head.
Everything here is float64 loops over taps with numpy array arithmetic: no blocking,
fusion or reordering beyond the definitions.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

# (name, cin, cout) of the 3x3x3 convolutions, in parameter order
LAYERS: List[Tuple[str, int, int]] = [
    ("e0a", 16, 16), ("e0b", 16, 16),      # level 0, down (16 input channels, 3 used)
    ("e1a", 16, 32), ("e1b", 32, 32),      # level 1, down
    ("b2a", 32, 64), ("b2b", 64, 64),      # level 2 (bottom)
    ("d1a", 96, 32), ("d1b", 32, 32),      # level 1, up: [upsampled 64 | skip 32]
    ("d0a", 48, 16), ("d0b", 16, 16),      # level 0, up: [upsampled 32 | skip 16]
]
HEAD_CIN = 16
IN_CHANNELS = 16          # input tensor channels; channels 3..15 are zero
P_SCALE = 0.2             # C/m^2
DOPING_SCALE = 1e24       # m^-3
V_SCALE = 2.0             # V
PHI_SCALE = 1.0           # V


def num_params() -> int:
    return sum(27 * ci * co + co for _, ci, co in LAYERS) + HEAD_CIN + 1


def unpack(theta: np.ndarray) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    """Views of the flat parameter vector: {layer: (W[27, cout, cin], b[cout])}."""
    out = {}
    o = 0
    for name, ci, co in LAYERS:
        W = theta[o:o + 27 * co * ci].reshape(27, co, ci)
        o += 27 * co * ci
        b = theta[o:o + co]
        o += co
        out[name] = (W, b)
    out["head"] = (theta[o:o + HEAD_CIN], theta[o + HEAD_CIN:o + HEAD_CIN + 1])
    assert o + HEAD_CIN + 1 == theta.size
    return out


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (fan-in 27 cin), zero biases; head weights scaled by 1/4."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in LAYERS:
        parts.append(rng.standard_normal(27 * co * ci) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(HEAD_CIN) * 0.25 * np.sqrt(1.0 / HEAD_CIN))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float64)


# --------------------------------------------------------------------- the ops
def taps():
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yield (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), dz, dy, dx


def shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[z, y, x] = x[z+dz, (y+dy) mod H, (x+dx) mod W], zero where z+dz is outside."""
    s = np.roll(x, shift=(-dy, -dx), axis=(1, 2))
    out = np.zeros_like(s)
    D = x.shape[0]
    if dz == 0:
        out[:] = s
    elif dz > 0:
        out[:D - dz] = s[dz:]
    else:
        out[-dz:] = s[:D + dz]
    return out


def shift_adjoint(g: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """Adjoint of shift(., dz, dy, dx): <shift(x), g> = <x, shift_adjoint(g)>."""
    out = np.zeros_like(g)
    D = g.shape[0]
    if dz == 0:
        out[:] = g
    elif dz > 0:
        out[dz:] = g[:D - dz]
    else:
        out[:D + dz] = g[-dz:]
    return np.roll(out, shift=(dy, dx), axis=(1, 2))


def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[v, o] = b[o] + sum over taps t and channels c of W[t, o, c] x[v + d_t, c]."""
    y = np.zeros(x.shape[:3] + (W.shape[1],)) + b
    for t, dz, dy, dx in taps():
        y += shift(x, dz, dy, dx) @ W[t].T
    return y


def conv3_backward(x: np.ndarray, W: np.ndarray, gz: np.ndarray):
    """Gradients of conv3 w.r.t. its input, weights and bias, given the output gradient gz."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, dz, dy, dx in taps():
        xs = shift(x, dz, dy, dx)
        gW[t] = np.einsum("zyxo,zyxc->oc", gz, xs)
        gx += shift_adjoint(gz @ W[t], dz, dy, dx)
    gb = gz.sum(axis=(0, 1, 2))
    return gx, gW, gb


def pool(x: np.ndarray) -> np.ndarray:
    """Mean over each 2x2x2 block."""
    D, H, Wd, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).mean(axis=(1, 3, 5))


def pool_backward(g: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(g, 2, 0), 2, 1), 2, 2) / 8.0


def up(x: np.ndarray) -> np.ndarray:
    """Each cell copied to its 2x2x2 children."""
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_backward(g: np.ndarray) -> np.ndarray:
    D, H, Wd, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).sum(axis=(1, 3, 5))


def relu(z):
    return np.maximum(z, 0.0)


# ----------------------------------------------------------------- the network
# Optional rounding hooks state a reduced-precision evaluation of the same network:
# `rnd` is applied to every stored activation (each convolution's ReLU output and each
# pooled tensor), `grnd` to every back-propagated signal entering a convolution's
# backward pass (after the ReLU mask).  Both default to none (plain float64).
def _id(v):
    return v


def forward(theta: np.ndarray, x: np.ndarray, keep: bool = False, rnd=None):
    """Network output (D, H, W) for input x (D, H, W, 16); with keep, also the activations."""
    rnd = rnd or _id
    p = unpack(theta)
    a = {}

    def layer(name, inp):
        W, b = p[name]
        out = rnd(relu(conv3(inp, W, b)))
        a[name + ".in"] = inp
        a[name] = out
        return out

    s0 = layer("e0b", layer("e0a", x))
    s1 = layer("e1b", layer("e1a", rnd(pool(s0))))
    bt = layer("b2b", layer("b2a", rnd(pool(s1))))
    c1 = np.concatenate([up(bt), s1], axis=3)
    u1 = layer("d1b", layer("d1a", c1))
    c0 = np.concatenate([up(u1), s0], axis=3)
    u0 = layer("d0b", layer("d0a", c0))
    w, b = p["head"]
    out = u0 @ w + b[0]
    return (out, a) if keep else out


def loss(theta: np.ndarray, x: np.ndarray, target: np.ndarray) -> float:
    """Mean squared error over all cells."""
    d = forward(theta, x) - target
    return float(np.mean(d * d))


def gradient(theta: np.ndarray, x: np.ndarray, target: np.ndarray, rnd=None, grnd=None, keep: bool = False):
    """(loss, d loss / d theta) by the chain rule through the layers above; with keep, also
    the signal entering each convolution's backward pass ({layer: dz})."""
    grnd = grnd or _id
    out, a = forward(theta, x, keep=True, rnd=rnd)
    p = unpack(theta)
    g = np.zeros_like(theta)
    gp = unpack(g)
    n = out.size
    d_out = 2.0 * (out - target) / n
    w, _ = p["head"]
    gw, gb = gp["head"]
    u0 = a["d0b"]
    gw[:] = np.einsum("zyx,zyxc->c", d_out, u0)
    gb[0] = d_out.sum()
    d = d_out[..., None] * w

    sig = {}

    def back(name, dy):
        W, _ = p[name]
        gW, gbb = gp[name]
        dz = grnd(dy * (a[name] > 0))
        sig[name] = dz
        dx, dW, db = conv3_backward(a[name + ".in"], W, dz)
        gW += dW
        gbb += db
        return dx

    d = back("d0a", back("d0b", d))                    # gradient w.r.t. c0 = [up(u1) | s0]
    c_up = a["d1b"].shape[3]
    d_u1 = up_backward(d[..., :c_up])
    d_s0 = d[..., c_up:].copy()
    d = back("d1a", back("d1b", d_u1))                 # w.r.t. c1 = [up(bt) | s1]
    c_up = a["b2b"].shape[3]
    d_bt = up_backward(d[..., :c_up])
    d_s1 = d[..., c_up:].copy()
    d = back("b2a", back("b2b", d_bt))                 # w.r.t. pool(s1)
    d_s1 += pool_backward(d)
    d = back("e1a", back("e1b", d_s1))                 # w.r.t. pool(s0)
    d_s0 += pool_backward(d)
    back("e0a", back("e0b", d_s0))
    L = float(np.mean((out - target) ** 2))
    return (L, g, sig) if keep else (L, g)


# --------------------------------------------------- inputs, targets, phi_lin
def phi_lin(spec, v_top: float) -> np.ndarray:
    """phi at the device-plane centres for P = 0 and no carriers: the layered series
    capacitor between the contacts (a constant D_z through resistances dz / eps_r)."""
    kb, kt = spec.device_range()
    eps = np.asarray(spec.plane_eps_r[kb:kt], np.float64)
    half = 0.5 / eps
    R_below = np.cumsum(np.concatenate([[0.0], 2 * half[:-1]])) + half    # bottom face -> centre k
    R_total = float(np.sum(1.0 / eps))
    return spec.v_bottom + (v_top - spec.v_bottom) * R_below / R_total


def pack_input(spec, P: np.ndarray, v_top: float) -> np.ndarray:
    """(nzd, ny, nx, 16): channel 0 P_z / P_SCALE, 1 (Nd - Na) / DOPING_SCALE per plane,
    2 V / V_SCALE everywhere, the rest zero."""
    kb, kt = spec.device_range()
    x = np.zeros((kt - kb, spec.ny, spec.nx, IN_CHANNELS))
    x[..., 0] = P[kb:kt] / P_SCALE
    dop = (np.asarray(spec.plane_Nd[kb:kt]) - np.asarray(spec.plane_Na[kb:kt])) / DOPING_SCALE
    x[..., 1] = dop[:, None, None]
    x[..., 2] = v_top / V_SCALE
    return x


def pack_target(spec, phi: np.ndarray, v_top: float) -> np.ndarray:
    """(phi - phi_lin(V)) / PHI_SCALE on the device planes."""
    kb, kt = spec.device_range()
    return (phi[kb:kt] - phi_lin(spec, v_top)[:, None, None]) / PHI_SCALE


def unpack_prediction(spec, out: np.ndarray, v_top: float) -> np.ndarray:
    """The starting iterate the prediction stands for, on the device planes."""
    return phi_lin(spec, v_top)[:, None, None] + PHI_SCALE * out
