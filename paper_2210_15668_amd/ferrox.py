"""Thin ctypes binding of libferrox.so (the HIP library); argument marshalling only.

Every step of the time step runs in the library's HIP kernels.  PyTorch is
used only to own device memory (the P and phi fields and the workspace) and
to supply the HIP stream.  If the library is missing this module raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libferrox.so")

FX_OK, FX_EINVAL, FX_ENOMEM, FX_EDEVICE, FX_ENOCONV, FX_ENONFINITE, FX_ESTATE = range(7)
FIELD_P, FIELD_PHI, FIELD_PHI_PREV, FIELD_PHI_PREV2, FIELD_PHI_PREV3 = 0, 1, 2, 3, 4
PROBE_OFF, PROBE_SMOOTH_FINE = 0, 1
LEVEL_LAUNCHES, LEVEL_BLOCKED, LEVEL_COARSE = 0, 1, 2
LAUNCH_STREAM, LAUNCH_GRAPH = 0, 1
TUNE_FORCE = 1
_STATUS = {0: "FX_OK", 1: "FX_EINVAL", 2: "FX_ENOMEM", 3: "FX_EDEVICE", 4: "FX_ENOCONV",
           5: "FX_ENONFINITE", 6: "FX_ESTATE"}


class FerroxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class StackDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double),
                ("plane_mat", ctypes.POINTER(ctypes.c_int)),
                ("plane_eps_r", ctypes.POINTER(ctypes.c_double)),
                ("plane_Na", ctypes.POINTER(ctypes.c_double)),
                ("plane_Nd", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("g11", ctypes.c_double), ("g44", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("pbc", ctypes.c_int), ("lam", ctypes.c_double),
                ("ni", ctypes.c_double), ("T", ctypes.c_double),
                ("v_bottom", ctypes.c_double), ("v_top", ctypes.c_double),
                ("tol_rel", ctypes.c_double), ("max_cycles", ctypes.c_int),
                ("prec", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("time_order", ctypes.c_int), ("carriers", ctypes.c_int),
                ("m_e", ctypes.c_double), ("m_p", ctypes.c_double), ("Eg", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("status", ctypes.c_int),
                ("res_norm", ctypes.c_double), ("rhs_norm", ctypes.c_double)]


class RunInfo(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int), ("total_cycles", ctypes.c_int),
                ("max_cycles_step", ctypes.c_int), ("last_res_rel", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps_done", ctypes.c_int), ("total_cycles", ctypes.c_int),
                ("max_cycles_step", ctypes.c_int), ("last_res_rel", ctypes.c_double)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("from_cache", ctypes.c_int), ("configs_timed", ctypes.c_int),
                ("cache_written", ctypes.c_int), ("default_us", ctypes.c_double), ("tuned_us", ctypes.c_double)]


# (name, restype, argtypes) of every entry point declared in include/ferrox.h
_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)
_D = ctypes.POINTER(StackDesc)
SIGNATURES = [
    ("stack_workspace_bytes", ctypes.c_size_t, [_D]),
    ("init_stack", ctypes.c_int, [_D, _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    ("poisson_solve_static", ctypes.c_int, [_D, _vp, _vp, _vp, ctypes.POINTER(SolveInfo)]),
    ("tdgl_step", ctypes.c_int, [_vp, ctypes.c_double]),
    ("poisson_solve", ctypes.c_int, [_vp, ctypes.c_double, ctypes.POINTER(SolveInfo)]),
    ("run_steps", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _dp, ctypes.POINTER(RunInfo)]),
    ("run_steps_qv", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, ctypes.POINTER(RunInfo)]),
    ("stack_qv", ctypes.c_int, [_vp, _dp, _dp]),
    ("get_field", ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    ("set_field", ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    ("stack_probe", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("stack_probe_read", ctypes.c_int, [_vp, _dp, _ip, _dp]),
    ("stack_num_levels", ctypes.c_int, [_vp]),
    ("stack_level_shape", ctypes.c_int, [_vp, ctypes.c_int, _ip, _ip, _ip]),
    ("stack_level_mode", ctypes.c_int, [_vp, ctypes.c_int, _ip]),
    ("destroy_stack", ctypes.c_int, [_vp]),
    ("stack_set_launch", ctypes.c_int, [_vp, ctypes.c_int]),
    ("stack_autotune", ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(TuneInfo)]),
    ("stack_tune_config", ctypes.c_int, [_vp, ctypes.c_int, _ip, _ip, _ip]),
    ("batch_autotune", ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(TuneInfo)]),
    # include/ferrox_unet.h
    ("unet_num_params", ctypes.c_size_t, []),
    ("unet_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("unet_init", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp,
                                 ctypes.POINTER(_vp)]),
    ("unet_set_params", ctypes.c_int, [_vp, _fp]),
    ("unet_get_params", ctypes.c_int, [_vp, _fp]),
    ("unet_pack_input", ctypes.c_int, [_vp, _vp, _dp, ctypes.c_double]),
    ("unet_set_input", ctypes.c_int, [_vp, _fp]),
    ("unet_get_input", ctypes.c_int, [_vp, _fp]),
    ("unet_forward", ctypes.c_int, [_vp, _vp]),
    ("unet_loss_grad", ctypes.c_int, [_vp, _vp, _dp, _fp]),
    ("unet_train_step", ctypes.c_int, [_vp, _vp, ctypes.c_float, _dp]),
    ("unet_destroy", ctypes.c_int, [_vp]),
    ("stack_unet_input", ctypes.c_int, [_vp, _vp, ctypes.c_double]),
    ("stack_unet_target", ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp]),
    ("stack_learned_solve", ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.POINTER(SolveInfo)]),
    ("batch_workspace_bytes", ctypes.c_size_t, [_D, ctypes.c_int]),
    ("init_batch", ctypes.c_int, [_D, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp,
                                  ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    ("run_batch", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_dp),
                                 ctypes.POINTER(BatchInfo)]),
    ("run_batch_qv", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                                    ctypes.POINTER(_dp), ctypes.POINTER(BatchInfo)]),
    ("batch_qv", ctypes.c_int, [_vp, _dp, _dp]),
    ("batch_get_field", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp]),
    ("batch_set_launch", ctypes.c_int, [_vp, ctypes.c_int]),
    ("batch_level_mode", ctypes.c_int, [_vp, ctypes.c_int, _ip]),
    ("destroy_batch", ctypes.c_int, [_vp]),
    ("last_error", ctypes.c_char_p, []),
]

_lib = None


def lib():
    """Load libferrox.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != FX_OK:
        raise FerroxError(status, lib().last_error().decode())


class _DescHolder:
    def __init__(self, spec: W.StackSpec):
        self.mat = np.ascontiguousarray(spec.plane_mat, np.int32)
        self.eps = np.ascontiguousarray(spec.plane_eps_r, np.float64)
        self.na = np.ascontiguousarray(spec.plane_Na, np.float64)
        self.nd = np.ascontiguousarray(spec.plane_Nd, np.float64)
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.d = StackDesc(spec.nx, spec.ny, spec.nz, spec.h,
                           self.mat.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           dp(self.eps), dp(self.na), dp(self.nd),
                           spec.alpha, spec.beta, spec.gamma, spec.g11, spec.g44, spec.Gamma,
                           spec.pbc, spec.lam, spec.ni, spec.T, spec.v_bottom, spec.v_top,
                           spec.tol_rel, spec.max_cycles, spec.prec, spec.warm_start,
                           spec.time_order, spec.carriers, spec.m_e, spec.m_p, spec.Eg)


def workspace_bytes(spec: W.StackSpec) -> int:
    h = _DescHolder(spec)
    return int(lib().stack_workspace_bytes(ctypes.byref(h.d)))


def poisson_solve_static(spec: W.StackSpec, P, phi, stream=None, check: bool = True) -> SolveInfo:
    """init_stack's Step 0 through poisson_solve_static: P and phi are float64 CUDA tensors of
    shape (nz, ny, nx) (P's entries off the ferroelectric are zeroed, phi receives the root);
    the library's static device workspace is used, nothing is allocated."""
    import torch
    shape = (spec.nz, spec.ny, spec.nx)
    for t in (P, phi):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and tuple(t.shape) == shape):
            raise ValueError("P and phi must be contiguous float64 CUDA tensors of shape (nz, ny, nx)")
    h = _DescHolder(spec)
    st = stream if stream is not None else torch.cuda.current_stream(P.device)
    info = SolveInfo()
    status = lib().poisson_solve_static(ctypes.byref(h.d), P.data_ptr(), phi.data_ptr(), st.cuda_stream,
                                        ctypes.byref(info))
    if check:
        _check(status)
    return info


class _Workspace:
    """The caller-owned workspace as a torch uint8 buffer; with guard > 0 (a multiple of
    256 bytes) it sits between two guard regions filled with 0xA5, which `intact()`
    checks (the library must never write outside the bytes it asked for)."""

    def __init__(self, torch, nbytes: int, device, guard: int = 0):
        if guard % 256:
            raise ValueError("guard must be a multiple of 256 bytes")
        self.guard, self.nbytes = guard, nbytes
        self.buf = torch.empty(nbytes + 2 * guard, dtype=torch.uint8, device=device)
        if guard:
            self.buf[:guard].fill_(0xA5)
            self.buf[guard + nbytes:].fill_(0xA5)

    def ptr(self) -> int:
        return self.buf.data_ptr() + self.guard

    def intact(self) -> bool:
        if not self.guard:
            return True
        g = self.guard
        return bool((self.buf[:g] == 0xA5).all().item()) and bool((self.buf[g + self.nbytes:] == 0xA5).all().item())


class Stack:
    """One device stack: P, phi and the workspace live in torch CUDA tensors.

    Construction runs Step 0 (phi for P^0).  ``P`` and ``phi`` are float64
    tensors of shape (nz, ny, nx) that always hold the current state.
    """

    def __init__(self, spec: W.StackSpec, P0, device: str = "cuda:0", stream=None, check_init: bool = True,
                 guard: int = 0):
        import torch
        self._torch = torch
        self.spec = spec
        self.device = torch.device(device)
        shape = (spec.nz, spec.ny, spec.nx)
        if isinstance(P0, np.ndarray):
            self.P = torch.from_numpy(np.ascontiguousarray(P0, np.float64)).to(self.device)
        else:
            self.P = P0.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(self.P.shape) == shape, (self.P.shape, shape)
        self.phi = torch.zeros(shape, dtype=torch.float64, device=self.device)
        self._desc = _DescHolder(spec)
        nbytes = int(lib().stack_workspace_bytes(ctypes.byref(self._desc.d)))
        if nbytes == 0:
            raise FerroxError(FX_EINVAL, lib().last_error().decode())
        self._ws = _Workspace(torch, nbytes, self.device, guard)
        self.ws = self._ws.buf
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = lib().init_stack(ctypes.byref(self._desc.d), self.P.data_ptr(), self.phi.data_ptr(),
                              self._ws.ptr(), nbytes, self.stream.cuda_stream, ctypes.byref(self._h))
        if not self._h.value:
            _check(st)
        self.init_status = st
        if check_init:
            _check(st)

    # ---------------------------------------------------------------- API
    def tdgl_step(self, dt: float):
        _check(lib().tdgl_step(self._h, dt))

    def poisson_solve(self, v_top: Optional[float] = None, check: bool = True) -> SolveInfo:
        info = SolveInfo()
        v = self.spec.v_top if v_top is None else v_top
        st = lib().poisson_solve(self._h, v, ctypes.byref(info))
        if check:
            _check(st)
        return info

    def run_steps(self, nsteps: int, dt: float, v_sched: Optional[Sequence[float]] = None,
                  check: bool = True) -> RunInfo:
        info = RunInfo()
        vs = None
        if v_sched is not None:
            self._vs = np.ascontiguousarray(v_sched, np.float64)
            assert len(self._vs) >= nsteps
            vs = self._vs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st = lib().run_steps(self._h, nsteps, dt, vs, ctypes.byref(info))
        if check:
            _check(st)
        return info

    def run_steps_qv(self, nsteps: int, dt: float, v_sched: Optional[Sequence[float]] = None,
                     check: bool = True):
        """run_steps that also returns Q [C/m^2] and V_fe [V] after every step: (info, Q, V_fe)."""
        info = RunInfo()
        vs = None
        if v_sched is not None:
            self._vs = np.ascontiguousarray(v_sched, np.float64)
            assert len(self._vs) >= nsteps
            vs = self._vs.ctypes.data_as(_dp)
        q = np.full(nsteps, np.nan)
        v = np.full(nsteps, np.nan)
        st = lib().run_steps_qv(self._h, nsteps, dt, vs, q.ctypes.data_as(_dp), v.ctypes.data_as(_dp),
                                ctypes.byref(info))
        if check:
            _check(st)
        return info, q, v

    def qv(self):
        """(Q [C/m^2], V_fe [V]) of the current state."""
        q, v = ctypes.c_double(), ctypes.c_double()
        _check(lib().stack_qv(self._h, ctypes.byref(q), ctypes.byref(v)))
        return q.value, v.value

    def get(self, which: int) -> np.ndarray:
        out = np.empty((self.spec.nz, self.spec.ny, self.spec.nx), np.float64)
        _check(lib().get_field(self._h, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set(self, which: int, arr: np.ndarray):
        a = np.ascontiguousarray(arr, np.float64)
        _check(lib().set_field(self._h, which, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def set_launch(self, mode: int):
        """LAUNCH_STREAM or LAUNCH_GRAPH for run_steps (see include/ferrox.h)."""
        _check(lib().stack_set_launch(self._h, mode))

    def autotune(self, cache_path: Optional[str] = None, force: bool = False) -> TuneInfo:
        """Time the smoother's launch shapes per level and keep the fastest (see include/ferrox.h)."""
        info = TuneInfo()
        path = cache_path.encode() if cache_path else None
        _check(lib().stack_autotune(self._h, path, TUNE_FORCE if force else 0, ctypes.byref(info)))
        return info

    def tune_config(self, level: int):
        """(tile width in threads, planes per thread, 8-wave register budget) in use at a level."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().stack_tune_config(self._h, level, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def probe(self, kernel: int = PROBE_SMOOTH_FINE, max_launches: int = 4096, stride: int = 1):
        """Start timestamping every stride-th finest-level smoother launch (see include/ferrox.h)."""
        _check(lib().stack_probe(self._h, kernel, max_launches, stride))

    def probe_read(self):
        """(total ms, launches, algorithmic bytes) of the probed launches."""
        ms, n, b = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
        _check(lib().stack_probe_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def levels(self):
        out = []
        for l in range(lib().stack_num_levels(self._h)):
            a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            _check(lib().stack_level_shape(self._h, l, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
            out.append((a.value, b.value, c.value))
        return out

    def level_modes(self):
        """Per level: LEVEL_LAUNCHES, LEVEL_BLOCKED or LEVEL_COARSE (how it is smoothed)."""
        out = []
        for l in range(lib().stack_num_levels(self._h)):
            m = ctypes.c_int()
            _check(lib().stack_level_mode(self._h, l, ctypes.byref(m)))
            out.append(m.value)
        return out

    def guard_intact(self) -> bool:
        """The guard regions around the workspace still hold their fill (see _Workspace)."""
        return self._ws.intact()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().destroy_stack(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(specs: Sequence[W.StackSpec]) -> int:
    hs = [_DescHolder(sp) for sp in specs]
    arr = (StackDesc * len(hs))(*[h.d for h in hs])
    return int(lib().batch_workspace_bytes(arr, len(hs)))


class Batch:
    """Independent stacks of different sizes advanced together (one launch per
    kernel for all of them).  ``P[i]`` and ``phi[i]`` are the instances'
    float64 tensors of shape (nz, ny, nx), holding the current state after
    every call.  Construction runs Step 0 for every instance."""

    def __init__(self, specs: Sequence[W.StackSpec], P0s, device: str = "cuda:0", stream=None,
                 check_init: bool = True, guard: int = 0):
        import torch
        self.specs = list(specs)
        self.n = len(self.specs)
        self.device = torch.device(device)
        self.P, self.phi = [], []
        for sp, P0 in zip(self.specs, P0s):
            shape = (sp.nz, sp.ny, sp.nx)
            if isinstance(P0, np.ndarray):
                P = torch.from_numpy(np.ascontiguousarray(P0, np.float64)).to(self.device)
            else:
                P = P0.to(device=self.device, dtype=torch.float64).contiguous()
            assert tuple(P.shape) == shape, (P.shape, shape)
            self.P.append(P)
            self.phi.append(torch.zeros(shape, dtype=torch.float64, device=self.device))
        self._hs = [_DescHolder(sp) for sp in self.specs]
        self._descs = (StackDesc * self.n)(*[h.d for h in self._hs])
        nbytes = int(lib().batch_workspace_bytes(self._descs, self.n))
        if nbytes == 0:
            raise FerroxError(FX_EINVAL, lib().last_error().decode())
        self._ws = _Workspace(torch, nbytes, self.device, guard)
        self.ws = self._ws.buf
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        pP = (_vp * self.n)(*[t.data_ptr() for t in self.P])
        pphi = (_vp * self.n)(*[t.data_ptr() for t in self.phi])
        self._h = ctypes.c_void_p()
        st = lib().init_batch(self._descs, self.n, pP, pphi, self._ws.ptr(), nbytes,
                              self.stream.cuda_stream, ctypes.byref(self._h))
        if not self._h.value:
            _check(st)
        self.init_status = st
        if check_init:
            _check(st)

    def run(self, nsteps: int, dt: float, v_scheds=None, check: bool = True):
        """nsteps time steps of every instance; returns a list of BatchInfo."""
        info = (BatchInfo * self.n)()
        vs = None
        if v_scheds is not None:
            self._vs = [np.ascontiguousarray(v, np.float64) for v in v_scheds]
            assert len(self._vs) == self.n and all(len(v) >= nsteps for v in self._vs)
            vs = (_dp * self.n)(*[v.ctypes.data_as(_dp) for v in self._vs])
        st = lib().run_batch(self._h, nsteps, dt, vs, info)
        if check:
            _check(st)
        return list(info)

    def run_qv(self, nsteps: int, dt: float, v_scheds=None, check: bool = True):
        """run that also records Q and V_fe after every step: (infos, Q[n][nsteps], V_fe[n][nsteps])."""
        info = (BatchInfo * self.n)()
        vs = None
        if v_scheds is not None:
            self._vs = [np.ascontiguousarray(v, np.float64) for v in v_scheds]
            assert len(self._vs) == self.n and all(len(v) >= nsteps for v in self._vs)
            vs = (_dp * self.n)(*[v.ctypes.data_as(_dp) for v in self._vs])
        q = [np.full(nsteps, np.nan) for _ in range(self.n)]
        v = [np.full(nsteps, np.nan) for _ in range(self.n)]
        pq = (_dp * self.n)(*[a.ctypes.data_as(_dp) for a in q])
        pv = (_dp * self.n)(*[a.ctypes.data_as(_dp) for a in v])
        st = lib().run_batch_qv(self._h, nsteps, dt, vs, pq, pv, info)
        if check:
            _check(st)
        return list(info), q, v

    def qv(self):
        """Arrays (Q, V_fe) of every instance's current state (NaN without an interface)."""
        q = np.empty(self.n)
        v = np.empty(self.n)
        _check(lib().batch_qv(self._h, q.ctypes.data_as(_dp), v.ctypes.data_as(_dp)))
        return q, v

    def get(self, inst: int, which: int) -> np.ndarray:
        sp = self.specs[inst]
        out = np.empty((sp.nz, sp.ny, sp.nx), np.float64)
        _check(lib().batch_get_field(self._h, inst, which, out.ctypes.data_as(_dp)))
        return out

    def set_launch(self, mode: int):
        _check(lib().batch_set_launch(self._h, mode))

    def level_modes(self, levels: int = 8):
        """LEVEL_LAUNCHES, LEVEL_BLOCKED or LEVEL_COARSE for levels 0 .. levels-1."""
        out = []
        for l in range(levels):
            m = ctypes.c_int()
            _check(lib().batch_level_mode(self._h, l, ctypes.byref(m)))
            out.append(m.value)
        return out

    def autotune(self, cache_path: Optional[str] = None, force: bool = False) -> TuneInfo:
        info = TuneInfo()
        path = cache_path.encode() if cache_path else None
        _check(lib().batch_autotune(self._h, path, TUNE_FORCE if force else 0, ctypes.byref(info)))
        return info

    def guard_intact(self) -> bool:
        """The guard regions around the workspace still hold their fill (see _Workspace)."""
        return self._ws.intact()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().destroy_batch(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UNet:
    """The learned warm start's network (include/ferrox_unet.h) over a stack's device slab
    of nzd x ny x nx cells.  Parameters are a flat float32 vector (unet_num_params())."""

    def __init__(self, nx: int, ny: int, nzd: int, train: bool = False, device: str = "cuda:0", stream=None):
        import torch
        self.shape = (nzd, ny, nx)
        self.device = torch.device(device)
        nbytes = int(lib().unet_workspace_bytes(nx, ny, nzd, 1 if train else 0))
        if nbytes == 0:
            raise FerroxError(FX_EINVAL, lib().last_error().decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        _check(lib().unet_init(nx, ny, nzd, 1 if train else 0, self.ws.data_ptr(), nbytes, self.stream.cuda_stream,
                               ctypes.byref(self._h)))
        self.nparams = int(lib().unet_num_params())

    @staticmethod
    def num_params() -> int:
        return int(lib().unet_num_params())

    def set_params(self, theta: np.ndarray):
        a = np.ascontiguousarray(theta, np.float32)
        assert a.size == self.nparams
        _check(lib().unet_set_params(self._h, a.ctypes.data_as(_fp)))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparams, np.float32)
        _check(lib().unet_get_params(self._h, a.ctypes.data_as(_fp)))
        return a

    def set_input(self, x: np.ndarray):
        a = np.ascontiguousarray(x, np.float32)
        assert a.shape == self.shape + (16,)
        _check(lib().unet_set_input(self._h, a.ctypes.data_as(_fp)))

    def get_input(self) -> np.ndarray:
        a = np.empty(self.shape + (16,), np.float32)
        _check(lib().unet_get_input(self._h, a.ctypes.data_as(_fp)))
        return a

    def pack_input(self, P_slab, doping_planes, v_top: float):
        """P_slab: float32 device tensor (nzd, ny, nx); doping_planes: nzd values of Nd - Na."""
        self._dop = np.ascontiguousarray(doping_planes, np.float64)
        _check(lib().unet_pack_input(self._h, P_slab.data_ptr(), self._dop.ctypes.data_as(_dp), float(v_top)))

    def forward(self, out=None, copy: bool = True):
        """Runs the network on its current input; returns a float32 tensor (nzd, ny, nx).
        With copy=False the output stays in the workspace (as in a learned solve, which
        places it into phi directly) and None is returned."""
        import torch
        if not copy:
            _check(lib().unet_forward(self._h, None))
            return None
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _check(lib().unet_forward(self._h, out.data_ptr()))
        return out

    def loss_grad(self, target, want_grad: bool = True):
        loss = ctypes.c_double()
        g = np.empty(self.nparams, np.float32) if want_grad else None
        _check(lib().unet_loss_grad(self._h, target.data_ptr(), ctypes.byref(loss),
                                    g.ctypes.data_as(_fp) if g is not None else None))
        return loss.value, g

    def train_step(self, target, lr: float, want_loss: bool = False):
        loss = ctypes.c_double()
        _check(lib().unet_train_step(self._h, target.data_ptr(), float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def input_from_stack(self, stack: "Stack", v_top: float):
        _check(lib().stack_unet_input(stack._h, self._h, float(v_top)))

    def target_from_stack(self, stack: "Stack", v_top: float, out=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _check(lib().stack_unet_target(stack._h, self._h, float(v_top), out.data_ptr()))
        return out

    def learned_solve(self, stack: "Stack", v_top: float, check: bool = True) -> SolveInfo:
        info = SolveInfo()
        st = lib().stack_learned_solve(stack._h, self._h, float(v_top), ctypes.byref(info))
        if check:
            _check(st)
        return info

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().unet_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
