"""MI355X-native anti-diagonal wavefront sweep (gfx950 HIP kernels behind a C ABI).

The Python layer only marshals arguments: every step of the sweep runs in libwf.so's
kernels.  PyTorch provides device memory and the current stream.  If libwf.so is missing
the calls raise; there is no CPU fallback.

Reading R0 of the cell recurrence (the paper does not state one):
    D[i][j] = C[i][j] + min(D[i-1][j-1], D[i-1][j], D[i][j-1]),
    virtual D[-1][-1] = 0, other virtual cells +inf;  score = D[m-1][n-1].
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import WfError  # noqa: F401

__all__ = ["forward", "ckpt_elems", "set_tile", "last_async_error", "WfError", "BAND"]

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
                        score.data_ptr(), ckpt.data_ptr() if ckpt is not None else None, ckpt_k,
                        _stream(C.device))
    _lib.check(rc, "wf_forward")
    return D, score, ckpt


def set_tile(tile: int) -> None:
    _lib.check(_lib.load().wf_set_tile(tile), "wf_set_tile")


def last_async_error(device=None) -> None:
    """Synchronizes the current stream and raises WfError if a device-side wait expired."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    _lib.check(_lib.load().wf_last_async_error(_stream(dev)), "device")
