"""MI355X-native anti-diagonal wavefront sweep (gfx950 HIP kernels behind a C ABI).

The Python layer only marshals arguments: every step of the sweep runs in libwf.so's
kernels.  PyTorch provides device memory and the current stream.  If libwf.so is missing
the calls raise; there is no CPU fallback.

Reading R0 of the cell recurrence (the paper does not state one):
    D[i][j] = C[i][j] + min(D[i-1][j-1], D[i-1][j], D[i][j-1]),
    virtual D[-1][-1] = 0, other virtual cells +inf;  score = D[m-1][n-1].
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import WfError  # noqa: F401

__all__ = ["forward", "backward", "sweep", "WfFunction", "Plan", "ckpt_elems", "set_tile", "predict_tile",
           "last_async_error", "WfError", "BAND", "soft_forward", "soft_backward", "soft_sweep", "SoftWfFunction"]

BAND = 64  # rows per band of the device sweep (= wavefront size)

_DTYPES = {torch.float32: _lib.WF_F32, torch.float64: _lib.WF_F64, torch.int32: _lib.WF_I32}


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return _DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}; use float32, float64 or int32") from None


def _check_matrix(C: torch.Tensor) -> None:
    if not C.is_cuda:
        raise ValueError("C must be a device tensor")
    if C.dim() != 2 or C.stride(1) != 1:
        raise ValueError("C must be a 2-D row-major tensor (unit column stride)")


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def ckpt_elems(m: int, n: int, ckpt_k: int) -> int:
    k = _lib.load().wf_ckpt_elems(m, n, ckpt_k)
    if k < 0:
        raise ValueError("invalid checkpoint configuration")
    return k


def forward(C: torch.Tensor, table: bool = True, ckpt_k: int = 0, D: torch.Tensor | None = None):
    """Forward sweep of one m x n instance on C's device and current stream.

    Returns (D, score, ckpt): D is the m x n table (None when table=False and no D was
    given), score a 0-d tensor, ckpt the checkpoint grid (None when ckpt_k == 0)."""
    _check_matrix(C)
    lib = _lib.load()
    m, n = C.shape
    if D is None and table:
        D = torch.empty((m, n), dtype=C.dtype, device=C.device)
    if D is not None:
        if D.shape != (m, n) or D.dtype != C.dtype or D.device != C.device or D.stride(1) != 1:
            raise ValueError("D must match C's shape, dtype and device, row-major")
    score = torch.empty((), dtype=C.dtype, device=C.device)
    ckpt = None
    if ckpt_k:
        ckpt = torch.empty(ckpt_elems(m, n, ckpt_k), dtype=C.dtype, device=C.device)
    rc = lib.wf_forward(_dtype_code(C), m, n, C.data_ptr(), C.stride(0),
                        D.data_ptr() if D is not None else None, D.stride(0) if D is not None else n,
                        score.data_ptr(), (ckpt.data_ptr() or None) if ckpt is not None else None, ckpt_k,
                        _stream(C.device))
    _lib.check(rc, "wf_forward")
    return D, score, ckpt


def backward(C: torch.Tensor, g_score: torch.Tensor | None = None, g_D: torch.Tensor | None = None,
             ckpt: torch.Tensor | None = None, ckpt_k: int = 0, D: torch.Tensor | None = None,
             g_C: torch.Tensor | None = None) -> torch.Tensor:
    """Adjoint sweep: returns g_C = dL/dC for L = sum(g_D * D) + g_score * score.

    The selections are recomputed on the device from C and either the checkpoint grid of
    forward(C, ckpt_k=K) (pass ckpt and ckpt_k=K) or the saved table D (exactly one)."""
    _check_matrix(C)
    lib = _lib.load()
    m, n = C.shape
    if (ckpt is None) == (D is None) or (ckpt is not None and ckpt_k < 1):
        raise ValueError("pass exactly one of ckpt (with ckpt_k) or D")
    for name, t in (("g_D", g_D), ("D", D), ("g_C", g_C)):
        if t is not None and (t.shape != (m, n) or t.dtype != C.dtype or t.device != C.device
                              or t.stride(1) != 1):
            raise ValueError(f"{name} must match C's shape, dtype and device, row-major")
    if ckpt is not None:
        if ckpt.dtype != C.dtype or ckpt.device != C.device or not ckpt.is_contiguous() \
                or ckpt.numel() != ckpt_elems(m, n, ckpt_k):
            raise ValueError("ckpt must be the checkpoint grid of forward(C, ckpt_k=ckpt_k)")
    if g_score is not None:
        g_score = g_score.to(device=C.device, dtype=C.dtype).reshape(()).contiguous()
    if g_C is None:
        g_C = torch.empty((m, n), dtype=C.dtype, device=C.device)
    rc = lib.wf_backward(_dtype_code(C), m, n, C.data_ptr(), C.stride(0),
                         (ckpt.data_ptr() or None) if ckpt is not None else None,
                         ckpt_k if ckpt is not None else 0,
                         D.data_ptr() if D is not None else None, D.stride(0) if D is not None else n,
                         g_score.data_ptr() if g_score is not None else None,
                         g_D.data_ptr() if g_D is not None else None, g_D.stride(0) if g_D is not None else n,
                         g_C.data_ptr(), g_C.stride(0), _stream(C.device))
    _lib.check(rc, "wf_backward")
    return g_C


def select(C: torch.Tensor, ckpt: torch.Tensor | None = None, ckpt_k: int = 0,
           D: torch.Tensor | None = None) -> None:
    """First half of backward: recomputes the predecessor selections of C's forward sweep
    into the device workspace (wf_select); reverse() then consumes them."""
    _check_matrix(C)
    m, n = C.shape
    if (ckpt is None) == (D is None) or (ckpt is not None and ckpt_k < 1):
        raise ValueError("pass exactly one of ckpt (with ckpt_k) or D")
    rc = _lib.load().wf_select(_dtype_code(C), m, n, C.data_ptr(), C.stride(0),
                               (ckpt.data_ptr() or None) if ckpt is not None else None,
                               ckpt_k if ckpt is not None else 0,
                               D.data_ptr() if D is not None else None, D.stride(0) if D is not None else n,
                               _stream(C.device))
    _lib.check(rc, "wf_select")


def reverse(m: int, n: int, dtype: torch.dtype = torch.float32, g_score: torch.Tensor | None = None,
            g_D: torch.Tensor | None = None, g_C: torch.Tensor | None = None, device=None) -> torch.Tensor:
    """Second half of backward: the reverse sweep from the selections of the last select()
    of this shape on the device (wf_reverse); returns g_C."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    if g_score is not None:
        g_score = g_score.to(device=dev, dtype=dtype).reshape(()).contiguous()
    if g_C is None:
        g_C = torch.empty((m, n), dtype=dtype, device=dev)
    code = {torch.float32: _lib.WF_F32, torch.float64: _lib.WF_F64, torch.int32: _lib.WF_I32}.get(dtype, -1)
    rc = _lib.load().wf_reverse(code, m, n, g_score.data_ptr() if g_score is not None else None,
                                g_D.data_ptr() if g_D is not None else None, g_D.stride(0) if g_D is not None else n,
                                g_C.data_ptr(), g_C.stride(0), _stream(dev))
    _lib.check(rc, "wf_reverse")
    return g_C


class WfFunction(torch.autograd.Function):
    """Differentiable sweep: (D, score) = sweep(C), gradient by the adjoint sweep.

    C is one m x n instance or a batch (B, m, n) of equal-size instances (swept together by
    one persistent launch per direction through a batch plan).  With table=False only the
    score(s) are produced and the forward keeps the checkpoint grid (band rows every 64
    rows, block columns every ckpt_k columns) instead of the table; with table=True the table
    is saved and the backward recomputes the selections from it."""

    @staticmethod
    def forward(ctx, C: torch.Tensor, table: bool, ckpt_k: int):
        C = C.contiguous()
        ctx.table = table
        # an output the loss does not use arrives as None, not as zeros: with the table's
        # gradient absent the adjoint of the score is the argmin path (wf_backward)
        ctx.set_materialize_grads(False)
        if C.dim() == 3:
            plan = _batch_plan(C)
            flat = C.view(-1)
            if table:
                scores, D, _ = plan.forward_ckpt(flat, 0, table=True)
                ctx.save_for_backward(C, D)
                ctx.plan = plan
                return D.view(C.shape), scores
            scores, _, ck = plan.forward_ckpt(flat, ckpt_k)
            ctx.save_for_backward(C, ck)
            ctx.plan, ctx.ckpt_k = plan, ckpt_k
            return scores
        if table:
            D, score, _ = forward(C, table=True)
            ctx.save_for_backward(C, D)
            return D, score
        _, score, ckpt = forward(C, table=False, ckpt_k=ckpt_k)
        ctx.save_for_backward(C, ckpt)
        ctx.ckpt_k = ckpt_k
        return score

    @staticmethod
    def backward(ctx, *grads):
        C, saved = ctx.saved_tensors
        if ctx.table:
            g_D, g_score = grads
            g_D = None if g_D is None else g_D.contiguous()
        else:
            (g_score,) = grads
            g_D = None
        if C.dim() == 3:
            plan = ctx.plan
            gD = None if g_D is None else g_D.reshape(-1)
            if ctx.table:
                g_C = plan.backward(C.view(-1), g_scores=g_score, g_D=gD, D=saved.view(-1))
            else:
                g_C = plan.backward(C.view(-1), g_scores=g_score, ckpt=saved, ckpt_k=ctx.ckpt_k)
            return g_C.view(C.shape), None, None
        if ctx.table:
            g_C = backward(C, g_score=g_score, g_D=g_D, D=saved)
        else:
            g_C = backward(C, g_score=g_score, ckpt=saved, ckpt_k=ctx.ckpt_k)
        return g_C, None, None


def sweep(C: torch.Tensor, table: bool = False, ckpt_k: int = 64):
    """Autograd entry point: score (table=False) or (D, score) (table=True) of an m x n
    instance, or scores of shape (B,) (and D of shape (B, m, n)) of a batch (B, m, n).
    ckpt_k: column spacing of the checkpoint grid kept for the backward (table=False)."""
    if C.dim() not in (2, 3):
        raise ValueError("C must be (m, n) or (B, m, n)")
    if not table and not 1 <= ckpt_k <= 4096:
        raise ValueError("ckpt_k must be in [1, 4096]")
    return WfFunction.apply(C, table, ckpt_k)


# ------------------------------------------------------------------------------------------
# Smooth variant: the minimum replaced by the soft minimum of temperature gamma.

def soft_forward(C: torch.Tensor, gamma: float, D: torch.Tensor | None = None):
    """Forward sweep of the soft-min recurrence (wf_soft_forward): returns (D, score)."""
    _check_matrix(C)
    m, n = C.shape
    if D is None:
        D = torch.empty((m, n), dtype=C.dtype, device=C.device)
    elif D.shape != (m, n) or D.dtype != C.dtype or D.device != C.device or D.stride(1) != 1:
        raise ValueError("D must match C's shape, dtype and device, row-major")
    score = torch.empty((), dtype=C.dtype, device=C.device)
    rc = _lib.load().wf_soft_forward(_dtype_code(C), m, n, float(gamma), C.data_ptr(), C.stride(0), D.data_ptr(),
                                     D.stride(0), score.data_ptr(), _stream(C.device))
    _lib.check(rc, "wf_soft_forward")
    return D, score


def soft_backward(C: torch.Tensor, D: torch.Tensor, gamma: float, g_score: torch.Tensor | None = None,
                  g_D: torch.Tensor | None = None, g_C: torch.Tensor | None = None) -> torch.Tensor:
    """Adjoint of the soft-min sweep (wf_soft_backward): g_C for L = sum(g_D * D) + g_score * score."""
    _check_matrix(C)
    m, n = C.shape
    for name, t in (("D", D), ("g_D", g_D), ("g_C", g_C)):
        if t is not None and (t.shape != (m, n) or t.dtype != C.dtype or t.device != C.device or t.stride(1) != 1):
            raise ValueError(f"{name} must match C's shape, dtype and device, row-major")
    if g_score is not None:
        g_score = g_score.to(device=C.device, dtype=C.dtype).reshape(()).contiguous()
    if g_C is None:
        g_C = torch.empty((m, n), dtype=C.dtype, device=C.device)
    rc = _lib.load().wf_soft_backward(_dtype_code(C), m, n, float(gamma), C.data_ptr(), C.stride(0), D.data_ptr(),
                                      D.stride(0), g_score.data_ptr() if g_score is not None else None,
                                      g_D.data_ptr() if g_D is not None else None,
                                      g_D.stride(0) if g_D is not None else n, g_C.data_ptr(), g_C.stride(0),
                                      _stream(C.device))
    _lib.check(rc, "wf_soft_backward")
    return g_C


class SoftWfFunction(torch.autograd.Function):
    """Differentiable soft-min sweep: (D, score) = soft_sweep(C, gamma); the table is saved
    for the backward, which runs the adjoint sweep on the device."""

    @staticmethod
    def forward(ctx, C: torch.Tensor, gamma: float):
        C = C.contiguous()
        D, score = soft_forward(C, gamma)
        ctx.save_for_backward(C, D)
        ctx.gamma = gamma
        return D, score

    @staticmethod
    def backward(ctx, g_D, g_score):
        C, D = ctx.saved_tensors
        g_D = None if g_D is None else g_D.contiguous()
        return soft_backward(C, D, ctx.gamma, g_score=g_score, g_D=g_D), None


def soft_sweep(C: torch.Tensor, gamma: float):
    """Autograd entry point of the soft-min sweep: (D, score) of an m x n instance."""
    if C.dim() != 2:
        raise ValueError("C must be (m, n)")
    return SoftWfFunction.apply(C, gamma)


_PLANS: dict = {}


def _batch_plan(C: torch.Tensor) -> "Plan":
    """The batch plan of B equal m x n instances stored contiguously (instance b at element
    offset b*m*n), created once per (B, m, n, dtype, device) and kept."""
    B, m, n = C.shape
    key = (B, m, n, C.dtype, C.device)
    plan = _PLANS.get(key)
    if plan is None:
        plan = Plan([m] * B, [n] * B, dtype=C.dtype, offsets=[b * m * n for b in range(B)], device=C.device)
        _PLANS[key] = plan
    return plan


class Plan:
    """A ragged batch of independent instances swept by one persistent launch.

    ms, ns: instance sizes; offsets: element offsets in one packed buffer (None = packed in
    order with 256-byte aligned starts); tile / rows: 16/32/64 and 1/2, or 0 to autotune.
    forward(C) takes the packed device buffer and returns (scores, D) -- D is None unless
    table=True or a D buffer is given."""

    def __init__(self, ms, ns, dtype=torch.float32, offsets=None, tile: int = 0, rows: int = 0, device=None):
        if len(ms) != len(ns) or not len(ms):
            raise ValueError("ms and ns must be non-empty and of equal length")
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.batch = len(ms)
        self.ms, self.ns = [int(x) for x in ms], [int(x) for x in ns]
        lib = _lib.load()
        arr = ctypes.c_int64 * self.batch
        m_arr, n_arr = arr(*self.ms), arr(*self.ns)
        o_arr = arr(*[int(x) for x in offsets]) if offsets is not None else None
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib.wf_plan_create(ctypes.byref(self._h), _DTYPES[dtype] if dtype in _DTYPES else -1, self.batch,
                                    m_arr, n_arr, o_arr, tile, rows, _stream(self.device))
        _lib.check(rc, "wf_plan_create")
        self.elems = lib.wf_plan_elems(self._h)
        out = arr()
        _lib.check(lib.wf_plan_offsets(self._h, out), "wf_plan_offsets")
        self.offsets = list(out)
        t, r = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(lib.wf_plan_config(self._h, ctypes.byref(t), ctypes.byref(r)), "wf_plan_config")
        self.tile, self.rows = t.value, r.value

    def pack(self, mats) -> torch.Tensor:
        """Packs a list of m_i x n_i tensors into one device buffer of the plan's layout."""
        buf = torch.zeros(self.elems, dtype=self.dtype, device=self.device)
        for o, x in zip(self.offsets, mats):
            buf[o:o + x.numel()].copy_(x.reshape(-1))
        return buf

    def unpack(self, buf: torch.Tensor):
        return [buf[o:o + m * n].view(m, n) for o, m, n in zip(self.offsets, self.ms, self.ns)]

    def forward(self, C: torch.Tensor, table: bool = False, D: torch.Tensor | None = None,
                scores: torch.Tensor | None = None):
        if C.dtype != self.dtype or C.device != self.device or not C.is_contiguous() or C.numel() < self.elems:
            raise ValueError("C must be a contiguous device buffer of the plan's dtype holding plan.elems elements")
        if D is None and table:
            D = torch.empty(self.elems, dtype=self.dtype, device=self.device)
        if D is not None and (D.dtype != self.dtype or D.device != self.device or not D.is_contiguous()
                              or D.numel() < self.elems):
            raise ValueError("D must be a contiguous device buffer like C")
        if scores is None:
            scores = torch.empty(self.batch, dtype=self.dtype, device=self.device)
        rc = _lib.load().wf_batch_forward(self._h, C.data_ptr(), D.data_ptr() if D is not None else None,
                                          scores.data_ptr(), _stream(self.device))
        _lib.check(rc, "wf_batch_forward")
        return scores, D

    def ckpt_elems(self, ckpt_k: int) -> int:
        k = _lib.load().wf_plan_ckpt_elems(self._h, ckpt_k)
        if k < 0:
            raise ValueError("invalid checkpoint spacing")
        return k

    def ckpt_offsets(self, ckpt_k: int):
        out = (ctypes.c_int64 * self.batch)()
        _lib.check(_lib.load().wf_plan_ckpt_offsets(self._h, ckpt_k, out), "wf_plan_ckpt_offsets")
        return list(out)

    def _check_buf(self, name, t, n=None):
        n = self.elems if n is None else n
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be a contiguous device buffer of the plan's dtype holding {n} elements")

    def forward_ckpt(self, C: torch.Tensor, ckpt_k: int, table: bool = False, D: torch.Tensor | None = None,
                     scores: torch.Tensor | None = None, ckpt: torch.Tensor | None = None):
        """forward() that also writes every instance's checkpoint grid (ckpt_k > 0):
        returns (scores, D, ckpt), the grids at ckpt_offsets(ckpt_k) of one buffer."""
        self._check_buf("C", C)
        if D is None and table:
            D = torch.empty(self.elems, dtype=self.dtype, device=self.device)
        if D is not None:
            self._check_buf("D", D)
        if scores is None:
            scores = torch.empty(self.batch, dtype=self.dtype, device=self.device)
        if ckpt is None and ckpt_k > 0:
            ckpt = torch.empty(self.ckpt_elems(ckpt_k), dtype=self.dtype, device=self.device)
        if ckpt is not None:
            self._check_buf("ckpt", ckpt, self.ckpt_elems(ckpt_k))
        rc = _lib.load().wf_batch_forward_ckpt(self._h, C.data_ptr(), D.data_ptr() if D is not None else None,
                                               scores.data_ptr(), (ckpt.data_ptr() or None) if ckpt is not None
                                               else None, ckpt_k, _stream(self.device))
        _lib.check(rc, "wf_batch_forward_ckpt")
        return scores, D, ckpt

    def backward(self, C: torch.Tensor, g_scores: torch.Tensor | None = None, g_D: torch.Tensor | None = None,
                 ckpt: torch.Tensor | None = None, ckpt_k: int = 0, D: torch.Tensor | None = None,
                 g_C: torch.Tensor | None = None) -> torch.Tensor:
        """Batched adjoint (wf_batch_backward): g_C in the plan's layout for
        L = sum_i (sum(g_D_i * D_i) + g_scores[i] * score_i), the selections recomputed from C
        and either the checkpoint grids (ckpt, ckpt_k) or the saved tables D."""
        if (ckpt is None) == (D is None) or (ckpt is not None and ckpt_k < 1):
            raise ValueError("pass exactly one of ckpt (with ckpt_k) or D")
        self._check_buf("C", C)
        for name, t in (("D", D), ("g_D", g_D), ("g_C", g_C)):
            if t is not None:
                self._check_buf(name, t)
        if ckpt is not None:
            self._check_buf("ckpt", ckpt, self.ckpt_elems(ckpt_k))
        if g_scores is not None:
            g_scores = g_scores.to(device=self.device, dtype=self.dtype).reshape(-1).contiguous()
            if g_scores.numel() != self.batch:
                raise ValueError("g_scores must hold one value per instance")
        if g_C is None:
            g_C = torch.empty(self.elems, dtype=self.dtype, device=self.device)
        rc = _lib.load().wf_batch_backward(self._h, C.data_ptr(),
                                           (ckpt.data_ptr() or None) if ckpt is not None else None,
                                           ckpt_k if ckpt is not None else 0,
                                           D.data_ptr() if D is not None else None,
                                           g_scores.data_ptr() if g_scores is not None else None,
                                           g_D.data_ptr() if g_D is not None else None, g_C.data_ptr(),
                                           _stream(self.device))
        _lib.check(rc, "wf_batch_backward")
        return g_C

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().wf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_tile(tile: int) -> None:
    _lib.check(_lib.load().wf_set_tile(tile), "wf_set_tile")


def predict_tile(m: int, n: int, reverse: bool = False, dtype: torch.dtype = torch.float32) -> int:
    """The tile G the library picks for an m x n instance when none is forced: the fastest
    tile of the nearest shape (in log2 m, log2 n) of its MI355X timing table for that element
    type (wf_tile_predict)."""
    code = {torch.float32: _lib.WF_F32, torch.float64: _lib.WF_F64, torch.int32: _lib.WF_I32}.get(dtype, -1)
    t = _lib.load().wf_tile_predict(code, m, n, 1 if reverse else 0)
    if t not in (16, 32, 64):
        raise _lib.WfError(t, "wf_tile_predict")
    return t


def last_async_error(device=None) -> None:
    """Synchronizes the current stream and raises WfError if a device-side wait expired."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    _lib.check(_lib.load().wf_last_async_error(_stream(dev)), "device")
