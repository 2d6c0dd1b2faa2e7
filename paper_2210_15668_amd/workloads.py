"""Seeded synthetic workloads: layer stacks, plane tables and initial P fields.

This module holds the problem *inputs* only -- material parameters, the
per-plane material tables of a layered gate stack, and the seeded random
initial polarisation.  It contains none of the method's arithmetic (no
stencils, no carrier statistics, no solver), so that both the CPU oracle
(test infrastructure) and the HIP library consume identical inputs without
sharing any code of the method.

Material parameters follow the paper's Table 1 (Landau coefficients
alpha/beta/gamma, gradient coefficients g11=g44, permittivities, mobility
Gamma, grid spacing, extrapolation length lambda).  The gradient coefficient
and time step used by the synthetic workloads are 1e-10 V m^3/C and 1e-13 s.

Orientation: z points from the back contact (k = 0, potential v_bottom) to
the gate (k = nz-1, potential v_top = V_app).  Layer lists are given
top-down, gate first, as the paper describes its stacks (ferroelectric on
top, then dielectric, then semiconductor).  Grid planes not covered by the
listed layers are electrode metal split between the two z-ends (odd plane at
the bottom).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

METAL, FE, DE, SC = 0, 1, 2, 3
PBC_FREE, PBC_ZERO, PBC_LAMBDA = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
CARRIERS_BOLTZMANN, CARRIERS_FD = 0, 1

# Table 1 of the paper (SI units)
ALPHA = -2.5e9          # V m / C
BETA = 6.0e10           # V m^5 / C^3
GAMMA_L = 1.5e11        # V m^9 / C^5
G_GRAD = 1.0e-10        # V m^3 / C (g11 = g44) for the synthetic workloads
MOBILITY = 100.0        # Gamma
EPS_FE = 24.0
EPS_SIO2 = 3.9
EPS_AL2O3 = 10.0
EPS_SI = 11.7
H = 0.5e-9              # m
LAMBDA = 3.0e-9         # m
DT = 1.0e-13            # s


@dataclasses.dataclass
class StackSpec:
    """A layered device stack on a periodic-in-x/y cell-centred grid."""

    nx: int
    ny: int
    nz: int
    h: float
    plane_mat: np.ndarray        # int32[nz]
    plane_eps_r: np.ndarray      # float64[nz]
    plane_Na: np.ndarray         # float64[nz], m^-3
    plane_Nd: np.ndarray         # float64[nz], m^-3
    alpha: float = ALPHA
    beta: float = BETA
    gamma: float = GAMMA_L
    g11: float = G_GRAD
    g44: float = G_GRAD
    Gamma: float = MOBILITY
    pbc: int = PBC_LAMBDA
    lam: float = LAMBDA
    ni: float = 1.0e16
    T: float = 300.0
    v_bottom: float = 0.0
    v_top: float = 0.0
    tol_rel: float = 1e-10
    max_cycles: int = 60
    prec: int = PREC_FP64
    warm_start: int = 3          # extrapolation order of each step's starting iterate
    time_order: int = 1          # 1 forward Euler, 2 predictor-corrector (two solves per step)
    carriers: int = CARRIERS_BOLTZMANN
    m_e: float = 1.08            # Table 1: effective masses / free-electron mass (Fermi-Dirac)
    m_p: float = 0.81
    Eg: float = 1.12             # eV, silicon at 300 K (Fermi-Dirac)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def device_range(self) -> Tuple[int, int]:
        nm = np.nonzero(self.plane_mat != METAL)[0]
        return int(nm[0]), int(nm[-1]) + 1

    def fe_range(self) -> Tuple[int, int]:
        fe = np.nonzero(self.plane_mat == FE)[0]
        return int(fe[0]), int(fe[-1]) + 1

    def n_active(self) -> int:
        kb, kt = self.device_range()
        return self.nx * self.ny * (kt - kb)

    def n_fe(self) -> int:
        f0, f1 = self.fe_range()
        return self.nx * self.ny * (f1 - f0)

    def copy(self, **kw) -> "StackSpec":
        d = dataclasses.asdict(self)
        d.update(kw)
        for k in ("plane_mat", "plane_eps_r", "plane_Na", "plane_Nd"):
            d[k] = np.array(d[k], copy=True)
        return StackSpec(**d)


def layered(nx: int, ny: int, nz: int, layers_top_down: Sequence[Tuple[int, int, float, float]],
            h: float = H, **kw) -> StackSpec:
    """Build a stack from (material, planes, eps_r, Na) layers listed gate-first.

    Remaining planes become electrode metal, split between the two ends with
    the odd plane at the bottom.
    """
    used = sum(l[1] for l in layers_top_down)
    if used > nz:
        raise ValueError("layers exceed nz")
    n_metal = nz - used
    top_metal = n_metal // 2
    bot_metal = n_metal - top_metal
    mat = np.zeros(nz, np.int32)
    eps = np.ones(nz, np.float64)
    na = np.zeros(nz, np.float64)
    nd = np.zeros(nz, np.float64)
    k = nz - top_metal
    for (m, n, e, a) in layers_top_down:
        k -= n
        mat[k:k + n] = m
        eps[k:k + n] = e
        na[k:k + n] = a
    assert k == bot_metal
    return StackSpec(nx, ny, nz, h, mat, eps, na, nd, **kw)


def random_P(spec: StackSpec, seed: int, amp: float = 0.01) -> np.ndarray:
    """Uniform random P_z in [-amp, amp] on ferroelectric planes, zero elsewhere.

    Draw order: numpy default_rng(seed).uniform over (n_fe_planes, ny, nx) in C
    order, bottom ferroelectric plane first.  Returns a full-grid float64 array
    of shape (nz, ny, nx).
    """
    f0, f1 = spec.fe_range()
    rng = np.random.default_rng(seed)
    P = np.zeros((spec.nz, spec.ny, spec.nx), np.float64)
    P[f0:f1] = rng.uniform(-amp, amp, (f1 - f0, spec.ny, spec.nx))
    return P


# --------------------------------------------------------------------------
# The synthetic workloads (shapes and parameters of the paper's stacks)
# --------------------------------------------------------------------------

def mfim_small() -> StackSpec:
    """16x16x32 MFIM: FE 16 planes (eps 24) over DE 4 planes (eps 3.9), metal 6+6, 1 V gate."""
    return layered(16, 16, 32, [(FE, 16, EPS_FE, 0.0), (DE, 4, EPS_SIO2, 0.0)],
                   v_top=1.0, tol_rel=1e-10)


def mfim_ramp() -> StackSpec:
    """128x128x64 MFIM: FE 40 / DE 8 (eps 3.9), metal 8+8; gate ramped 0 -> 1.5 V over 2000 steps."""
    return layered(128, 128, 64, [(FE, 40, EPS_FE, 0.0), (DE, 8, EPS_SIO2, 0.0)],
                   v_top=0.0, tol_rel=1e-10)


def mfism_large(prec: int = PREC_FP64) -> StackSpec:
    """256x256x128 MFISM: FE 48 / SiO2 8 / p-Si 64 (Na 1e24, ni 1e16, 300 K), metal 4+4, 1 V gate."""
    return layered(256, 256, 128, [(FE, 48, EPS_FE, 0.0), (DE, 8, EPS_SIO2, 0.0),
                                   (SC, 64, EPS_SI, 1.0e24)],
                   v_top=1.0, ni=1.0e16, T=300.0, tol_rel=1e-10, prec=prec)


def mfism_medium(prec: int = PREC_FP64) -> StackSpec:
    """128x128x64 MFISM: FE 24 / SiO2 4 / p-Si 32, metal 2+2 (half of the large stack's proportions)."""
    return layered(128, 128, 64, [(FE, 24, EPS_FE, 0.0), (DE, 4, EPS_SIO2, 0.0),
                                  (SC, 32, EPS_SI, 1.0e24)],
                   v_top=1.0, ni=1.0e16, T=300.0, tol_rel=1e-10, prec=prec)


def convergence_mfism(n: int = 128, prec: int = PREC_FP64) -> StackSpec:
    """The MFISM cube of the paper's convergence study (Methods, numerical validation;
    Table 2): 32 nm on each side in n^3 cells, the bottom quarter undoped Si, the next
    quarter SiO2, the upper half ferroelectric; phi = 0 on both z-faces; the lambda = 3 nm
    surface condition; Table 1's gradient coefficient g11 = g44 = 1e-9 V m^3/C."""
    if n % 4:
        raise ValueError("n must be a multiple of 4")
    q = n // 4
    return layered(n, n, n, [(FE, 2 * q, EPS_FE, 0.0), (DE, q, EPS_SIO2, 0.0), (SC, q, EPS_SI, 0.0)],
                   h=32e-9 / n, g11=1.0e-9, g44=1.0e-9, v_top=0.0, v_bottom=0.0,
                   ni=1.0e16, T=300.0, tol_rel=1e-13, prec=prec)


def gaussian_bump_P(spec: StackSpec, amp: float = 0.002, sigma_xy: float = 5e-9,
                    sigma_z: float = 2e-9, z0: float = 24e-9) -> np.ndarray:
    """The convergence study's initial P: amp exp(-(x^2 + y^2)/(2 sigma_xy^2)
    - (z - z0)^2/(2 sigma_z^2)) on the ferroelectric planes, zero elsewhere.  z is the
    height of the cell centre above the bottom face; x and y are measured from the centre
    of the periodic footprint."""
    h = spec.h
    x = (np.arange(spec.nx) + 0.5) * h - 0.5 * spec.nx * h
    y = (np.arange(spec.ny) + 0.5) * h - 0.5 * spec.ny * h
    z = (np.arange(spec.nz) + 0.5) * h
    P = amp * np.exp(-(x[None, None, :] ** 2 + y[None, :, None] ** 2) / (2 * sigma_xy ** 2)
                     - (z[:, None, None] - z0) ** 2 / (2 * sigma_z ** 2))
    f0, f1 = spec.fe_range()
    P[:f0] = 0.0
    P[f1:] = 0.0
    return P


CONVERGENCE_DT = (50e-15, 25e-15, 12.5e-15)   # s: coarse, medium, fine time steps
CONVERGENCE_T_END = 400e-15                    # s


def shrink_lateral(spec: StackSpec, nx: int, ny: int) -> StackSpec:
    """Same z-stack on a smaller periodic x-y footprint (for oracle-sized parity cases)."""
    return spec.copy(nx=nx, ny=ny)


def ramp_schedule(nsteps: int, v_final: float = 1.5, n_ramp: int = 2000) -> np.ndarray:
    """Gate voltage for the solve producing phi^n, n = 1..nsteps: v_final * n / n_ramp."""
    n = np.arange(1, nsteps + 1, dtype=np.float64)
    return v_final * np.minimum(n, n_ramp) / n_ramp


def triangle_schedule(nsteps: int, v_max: float, period: int, v0: float = 0.0) -> np.ndarray:
    """Triangular gate wave for the solves producing phi^n, n = 1..nsteps: from v0 up to
    v0 + v_max at a quarter period, down to v0 - v_max at three quarters, back at a full
    period (the Q-V sweeps of the Results section)."""
    t = (np.arange(1, nsteps + 1, dtype=np.float64) / period) % 1.0
    w = np.where(t < 0.25, 4 * t, np.where(t < 0.75, 2 - 4 * t, 4 * t - 4))
    return v0 + v_max * w


def mfim_fig3(n_lateral: int = 64, prec: int = PREC_FP64) -> StackSpec:
    """The 3D MFIM of the Results (Q-V loops): 5 nm ferroelectric over 4 nm Al2O3, 32 nm
    lateral at h = 0.5 nm (64 x 64 cells; n_lateral shrinks the footprint), one metal plane
    at each end; Table 1's g11 = g44 = 1e-9 V m^3/C."""
    return layered(n_lateral, n_lateral, 20, [(FE, 10, EPS_FE, 0.0), (DE, 8, EPS_AL2O3, 0.0)],
                   g11=1.0e-9, g44=1.0e-9, v_top=0.0, tol_rel=1e-10, prec=prec)


DT_TABLE1 = 4.0e-13      # s, Table 1's time step (with g = 1e-9 and h = 0.5 nm)


def mfism_fig4(n_lateral: int = 64, prec: int = PREC_FP64) -> StackSpec:
    """The 3D MFISM of the Results (FeFET gate stack): 5 nm ferroelectric, 1 nm SiO2, 10 nm
    undoped silicon with Fermi-Dirac carriers (Table 1's effective masses), 32 nm lateral at
    h = 0.5 nm (64 x 64 cells; n_lateral shrinks the footprint), one metal plane at each end,
    0 V gate; Table 1's g11 = g44 = 1e-9 V m^3/C."""
    return layered(n_lateral, n_lateral, 34, [(FE, 10, EPS_FE, 0.0), (DE, 2, EPS_SIO2, 0.0),
                                              (SC, 20, EPS_SI, 0.0)],
                   g11=1.0e-9, g44=1.0e-9, v_top=0.0, T=300.0, carriers=CARRIERS_FD,
                   tol_rel=1e-10, prec=prec)


def batch_instances(count: int = 64, seed0: int = 100) -> List[Tuple[StackSpec, np.ndarray]]:
    """Uneven MFIM instances: x,y from {32,48,64,96}, z from {32,48}, FE 16..min(32,nz-4), DE 4.

    Each instance draws its sizes, gate voltage (uniform in [-2, 2] V) and
    initial P from default_rng(seed0 + index).
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        nx = int(rng.choice([32, 48, 64, 96]))
        ny = int(rng.choice([32, 48, 64, 96]))
        nz = int(rng.choice([32, 48]))
        nfe = int(rng.integers(16, min(32, nz - 4) + 1))
        v = float(rng.uniform(-2.0, 2.0))
        spec = layered(nx, ny, nz, [(FE, nfe, EPS_FE, 0.0), (DE, 4, EPS_SIO2, 0.0)], v_top=v)
        f0, f1 = spec.fe_range()
        P = np.zeros((nz, ny, nx))
        P[f0:f1] = rng.uniform(-0.01, 0.01, (f1 - f0, ny, nx))
        out.append((spec, P))
    return out
