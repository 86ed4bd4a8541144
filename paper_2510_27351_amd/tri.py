"""Tridiagonal partition solver on MI355X (include/tri.h).  Argument marshalling only.

A system is four device vectors a (sub-diagonal, a[0] unused), b (diagonal), c
(super-diagonal, c[N-1] unused), d (right-hand side): row i reads
a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i].  A batch is a (batch, N) tensor per array.
Every stage runs in libwf.so's kernels on the tensors' device and current stream; there is
no CPU path.

    stage1(a, b, c, d, m)        -> (A, B, C, D)   interface systems, (batch, 2P) each
    stage3(a, b, c, d, z, m)     -> x              solution from the interface unknowns z
    thomas(a, b, c, d)           -> x              direct solve (the deepest level's solver)
    Plan(batch, N, dtype, m, R, ms).solve(a, b, c, d) -> x
    solve(a, b, c, d, m=0, R=-1, ms=None)          -> x    (a plan per call)
    predict(N, dtype)            -> (m, R, ms)     the 1-NN choice timed on MI355X
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

TRI_MAX_R = 6

_DTYPES = {torch.float32: _lib.WF_F32, torch.float64: _lib.WF_F64}


def _code(dtype: torch.dtype) -> int:
    try:
        return _DTYPES[dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {dtype}; use float32 or float64") from None


def _system(*vs: torch.Tensor):
    """(batch, N) of a set of same-shaped, contiguous device tensors (1-D = one system)."""
    v0 = vs[0]
    for v in vs:
        if not v.is_cuda:
            raise ValueError("the system must be on a GPU device")
        if v.shape != v0.shape or v.dtype != v0.dtype or v.device != v0.device:
            raise ValueError("a, b, c, d must share shape, dtype and device")
        if not v.is_contiguous():
            raise ValueError("the arrays must be contiguous")
    if v0.dim() == 1:
        return 1, v0.shape[0]
    if v0.dim() == 2:
        return v0.shape[0], v0.shape[1]
    raise ValueError("expected (N,) or (batch, N) arrays")


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def subsystems(N: int, m: int) -> int:
    """Number of sub-systems of N rows cut into sub-systems of m rows."""
    P = _lib.load().tri_subsystems(N, m)
    if P < 0:
        raise ValueError("the partition needs N >= 2 and m >= 2")
    return P


def stage1(a, b, c, d, m: int):
    """Stage 1: the interface systems (A, B, C, D), each shaped like a with 2P columns."""
    batch, N = _system(a, b, c, d)
    P = subsystems(N, m)
    shape = (2 * P,) if a.dim() == 1 else (batch, 2 * P)
    out = [torch.empty(shape, dtype=a.dtype, device=a.device) for _ in range(4)]
    rc = _lib.load().tri_stage1(_code(a.dtype), batch, N, m, a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                d.data_ptr(), *(o.data_ptr() for o in out), _stream(a.device))
    _lib.check(rc, "tri_stage1")
    return tuple(out)


def stage3(a, b, c, d, z, m: int, x=None):
    """Stage 3: the solution from the interface unknowns z (shaped like the interface system)."""
    batch, N = _system(a, b, c, d)
    P = subsystems(N, m)
    if z.dtype != a.dtype or z.device != a.device or not z.is_contiguous() or z.numel() != batch * 2 * P:
        raise ValueError("z must hold 2P values per system, contiguous, of the system's dtype and device")
    if x is None:
        x = torch.empty_like(a)
    rc = _lib.load().tri_stage3(_code(a.dtype), batch, N, m, a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                d.data_ptr(), z.data_ptr(), x.data_ptr(), _stream(a.device))
    _lib.check(rc, "tri_stage3")
    return x


def thomas(a, b, c, d):
    """Direct solve of every system by the Thomas algorithm (one workgroup per system)."""
    batch, N = _system(a, b, c, d)
    x = torch.empty_like(a)
    scratch = torch.empty(2 * batch * N, dtype=a.dtype, device=a.device)
    rc = _lib.load().tri_thomas(_code(a.dtype), batch, N, a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                d.data_ptr(), x.data_ptr(), scratch.data_ptr(), _stream(a.device))
    _lib.check(rc, "tri_thomas")
    return x


def predict(N: int, dtype=torch.float64):
    """(m, R, [m_1 .. m_R]) predicted for a system of N unknowns."""
    m, R = ctypes.c_int32(), ctypes.c_int32()
    ms = (ctypes.c_int32 * TRI_MAX_R)()
    _lib.check(_lib.load().tri_predict(_code(dtype), N, ctypes.byref(m), ctypes.byref(R), ms), "tri_predict")
    return m.value, R.value, [ms[i] for i in range(R.value)]


class Plan:
    """The full solver for 'batch' systems of N unknowns (m = 0 / R = -1 / ms = None: the
    predictor's choice).  Owns the interface systems of every level on the current device."""

    def __init__(self, batch: int, N: int, dtype=torch.float64, m: int = 0, R: int = -1, ms=None):
        self._lib = _lib.load()
        self.batch, self.N, self.dtype = batch, N, dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        arr = None
        if ms is not None:
            arr = (ctypes.c_int32 * max(1, len(ms)))(*ms)
        h = ctypes.c_void_p()
        _lib.check(self._lib.tri_plan_create(ctypes.byref(h), _code(dtype), batch, N, m, R, arr), "tri_plan_create")
        self._h = h
        cm, cR = ctypes.c_int32(), ctypes.c_int32()
        cms = (ctypes.c_int32 * TRI_MAX_R)()
        sizes = (ctypes.c_int64 * (TRI_MAX_R + 2))()
        _lib.check(self._lib.tri_plan_config(h, ctypes.byref(cm), ctypes.byref(cR), cms, sizes), "tri_plan_config")
        self.m, self.R = cm.value, cR.value
        self.ms = [cms[i] for i in range(max(0, self.R))]
        self.sizes = [sizes[i] for i in range(self.R + 2)] if self.R >= 0 else [N]

    def solve(self, a, b, c, d, x=None):
        batch, N = _system(a, b, c, d)
        if (batch, N) != (self.batch, self.N) or a.dtype != self.dtype or a.device != self.device:
            raise ValueError("the system does not match the plan")
        if x is None:
            x = torch.empty_like(a)
        elif x.shape != a.shape or x.dtype != a.dtype or x.device != a.device or not x.is_contiguous():
            raise ValueError("x must match a")
        rc = self._lib.tri_solve(self._h, a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr(), x.data_ptr(),
                                 _stream(a.device))
        _lib.check(rc, "tri_solve")
        return x

    def level(self, l: int):
        """Level l's interface system (A, B, C, D) of the last solve, (batch, sizes[l]) each."""
        if not 1 <= l <= self.R + 1:
            raise ValueError("level out of range")
        out = [torch.empty((self.batch, self.sizes[l]), dtype=self.dtype, device=self.device) for _ in range(4)]
        rc = self._lib.tri_plan_level(self._h, l, *(o.data_ptr() for o in out), _stream(self.device))
        _lib.check(rc, "tri_plan_level")
        return tuple(out)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.tri_plan_destroy(h)
            self._h = None


def solve(a, b, c, d, m: int = 0, R: int = -1, ms=None):
    """x = A^-1 d by the partition method (a plan is made for the call)."""
    batch, N = _system(a, b, c, d)
    return Plan(batch, N, a.dtype, m, R, ms).solve(a, b, c, d)
