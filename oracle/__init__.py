"""CPU FP64 oracle of the TDGL + Poisson time step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never calls it, and
it shares no code with the HIP path: the C source ``ferro_oracle.c`` holds
every step of the method the oracle computes (see its header for the
discrete definition and the paper passages it follows).

Fields are numpy float64 arrays of shape (nz, ny, nx) (z-major, k = 0 at the
back contact), matching the ``StackSpec`` inputs of
``paper_2210_15668_amd.workloads``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ferro_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double),
                ("mat", ctypes.POINTER(ctypes.c_int)),
                ("eps_r", ctypes.POINTER(ctypes.c_double)),
                ("Na", ctypes.POINTER(ctypes.c_double)),
                ("Nd", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("g11", ctypes.c_double), ("g44", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("pbc", ctypes.c_int), ("lam", ctypes.c_double),
                ("ni", ctypes.c_double), ("T", ctypes.c_double),
                ("v_bottom", ctypes.c_double), ("v_top", ctypes.c_double),
                ("carriers", ctypes.c_int), ("me", ctypes.c_double), ("mp", ctypes.c_double),
                ("Eg", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("cg_iters", ctypes.c_int),
                ("res_norm", ctypes.c_double), ("rhs_norm", ctypes.c_double),
                ("status", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(_Desc)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_tdgl_rhs.argtypes = [D, dp, dp, dp]
        lib.orc_tdgl_step.argtypes = [D, dp, dp, ctypes.c_double, dp]
        lib.orc_solve.argtypes = [D, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)]
        lib.orc_poisson_parts.argtypes = [D, dp, dp, dp, dp, dp, dp]
        lib.orc_residual_norms.argtypes = [D, dp, dp, dp, dp]
        lib.orc_run.argtypes = [D, dp, dp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                ctypes.c_int, ctypes.POINTER(Info)]
        lib.orc_run_pc.argtypes = [D, dp, dp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                ctypes.c_int, ctypes.POINTER(Info)]
        lib.orc_qv.argtypes = [D, dp, dp, dp, dp]
        lib.orc_fd_half.argtypes = [ctypes.c_double, dp, dp]
        lib.orc_fd_half.restype = None
        lib.orc_plane_densities.argtypes = [D, ctypes.c_int, dp, dp]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _DescHolder:
    """Keeps the plane arrays alive for the lifetime of the ctypes struct."""

    def __init__(self, spec, v_top: Optional[float] = None):
        self.mat = np.ascontiguousarray(spec.plane_mat, dtype=np.int32)
        self.eps = np.ascontiguousarray(spec.plane_eps_r, dtype=np.float64)
        self.na = np.ascontiguousarray(spec.plane_Na, dtype=np.float64)
        self.nd = np.ascontiguousarray(spec.plane_Nd, dtype=np.float64)
        self.d = _Desc(spec.nx, spec.ny, spec.nz, spec.h,
                       self.mat.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       _ptr(self.eps), _ptr(self.na), _ptr(self.nd),
                       spec.alpha, spec.beta, spec.gamma, spec.g11, spec.g44, spec.Gamma,
                       spec.pbc, spec.lam, spec.ni, spec.T, spec.v_bottom,
                       spec.v_top if v_top is None else v_top,
                       spec.carriers, spec.m_e, spec.m_p, spec.Eg)

    @property
    def ref(self):
        return ctypes.byref(self.d)


def _shape(spec):
    return (spec.nz, spec.ny, spec.nx)


def tdgl_rhs(spec, P: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """f(P, phi) of the TDGL equation on ferroelectric cells."""
    lib = _load()
    h = _DescHolder(spec)
    P = np.ascontiguousarray(P, np.float64)
    phi = np.ascontiguousarray(phi, np.float64)
    out = np.zeros(_shape(spec))
    if lib.orc_tdgl_rhs(h.ref, _ptr(P), _ptr(phi), _ptr(out)):
        raise ValueError("invalid stack")
    return out


def tdgl_step(spec, P: np.ndarray, phi: np.ndarray, dt: float) -> np.ndarray:
    """Step 1a: P + dt f(P, phi)."""
    lib = _load()
    h = _DescHolder(spec)
    P = np.ascontiguousarray(P, np.float64)
    phi = np.ascontiguousarray(phi, np.float64)
    out = np.zeros(_shape(spec))
    if lib.orc_tdgl_step(h.ref, _ptr(P), _ptr(phi), dt, _ptr(out)):
        raise ValueError("invalid stack")
    return out


def solve(spec, P: np.ndarray, phi0: Optional[np.ndarray] = None, tol: float = 1e-13,
          max_newton: int = 200, v_top: Optional[float] = None, check: bool = True):
    """Solve the discrete Poisson problem for P; returns (phi, Info)."""
    lib = _load()
    h = _DescHolder(spec, v_top)
    P = np.ascontiguousarray(P, np.float64)
    phi = np.zeros(_shape(spec)) if phi0 is None else np.array(phi0, dtype=np.float64, copy=True)
    info = Info()
    s = lib.orc_solve(h.ref, _ptr(P), _ptr(phi), tol, max_newton, ctypes.byref(info))
    if check and s != 0:
        raise RuntimeError(f"oracle solve failed: status {s}, |r|={info.res_norm}, |f|={info.rhs_norm}")
    return phi, info


def poisson_parts(spec, P: np.ndarray, phi: np.ndarray, v_top: Optional[float] = None):
    """Returns (f, N(phi), rho_c(phi), sigma(phi)) on the full grid."""
    lib = _load()
    h = _DescHolder(spec, v_top)
    P = np.ascontiguousarray(P, np.float64)
    phi = np.ascontiguousarray(phi, np.float64)
    outs = [np.zeros(_shape(spec)) for _ in range(4)]
    if lib.orc_poisson_parts(h.ref, _ptr(P), _ptr(phi), *[_ptr(o) for o in outs]):
        raise ValueError("invalid stack")
    return tuple(outs)


def residual_norms(spec, P: np.ndarray, phi: np.ndarray, v_top: Optional[float] = None):
    """(||f - N(phi)||_2, ||f||_2) over device cells."""
    lib = _load()
    h = _DescHolder(spec, v_top)
    P = np.ascontiguousarray(P, np.float64)
    phi = np.ascontiguousarray(phi, np.float64)
    rn = ctypes.c_double()
    fn = ctypes.c_double()
    if lib.orc_residual_norms(h.ref, _ptr(P), _ptr(phi), ctypes.byref(rn), ctypes.byref(fn)):
        raise ValueError("invalid stack")
    return rn.value, fn.value


def fd_half(eta: float):
    """(F, dF/deta) of the Fermi-Dirac integral of order 1/2 as the oracle evaluates it."""
    lib = _load()
    F, dF = ctypes.c_double(), ctypes.c_double()
    lib.orc_fd_half(float(eta), ctypes.byref(F), ctypes.byref(dF))
    return F.value, dF.value


def plane_densities(spec, k: int):
    """(p0, n0): the neutral-bulk hole and electron densities of semiconductor plane k."""
    lib = _load()
    h = _DescHolder(spec)
    p0, n0 = ctypes.c_double(), ctypes.c_double()
    if lib.orc_plane_densities(h.ref, k, ctypes.byref(p0), ctypes.byref(n0)):
        raise ValueError("not a semiconductor plane")
    return p0.value, n0.value


def qv(spec, P: np.ndarray, phi: np.ndarray):
    """(Q, V_fe^avg) of the Q-V characteristics for the given fields (see orc_qv)."""
    lib = _load()
    h = _DescHolder(spec)
    Pc = np.ascontiguousarray(P, np.float64)
    pc = np.ascontiguousarray(phi, np.float64)
    q, v = ctypes.c_double(), ctypes.c_double()
    if lib.orc_qv(h.ref, _ptr(Pc), _ptr(pc), ctypes.byref(q), ctypes.byref(v)):
        raise ValueError("no ferroelectric/dielectric interface")
    return q.value, v.value


def run(spec, P0: np.ndarray, nsteps: int, dt: float, v_sched: Optional[Sequence[float]] = None,
        tol: float = 1e-13, phi0: Optional[np.ndarray] = None, max_newton: int = 200,
        init: bool = True, order: int = 1):
    """Step 0 (if ``init``) then ``nsteps`` steps of the forward-Euler scheme (order 1) or the
    predictor-corrector (order 2); returns (P, phi, Info of the last solve)."""
    lib = _load()
    P = np.array(P0, dtype=np.float64, copy=True)
    if init:
        phi, _ = solve(spec, P, None, tol, max_newton)
    else:
        phi = np.array(phi0, dtype=np.float64, copy=True)
    h = _DescHolder(spec)
    vs = None if v_sched is None else np.ascontiguousarray(v_sched, np.float64)
    info = Info()
    fn = lib.orc_run_pc if order == 2 else lib.orc_run
    s = fn(h.ref, _ptr(P), _ptr(phi), nsteps, dt, _ptr(vs), tol, max_newton, ctypes.byref(info))
    if s:
        raise RuntimeError(f"oracle run failed: status {s}")
    return P, phi, info
