"""CPU oracle for the wavefront cell recurrence -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product library never imports, links or calls it, and it shares
no code with the GPU path (the only shared module is the seeded input generator, which holds
none of the method's arithmetic).

The arithmetic lives in ``wf_oracle.c`` (plain row-by-row C, -O2, no fast-math, no FP
contraction); this module only marshals numpy arrays.  See that file's header for the
recurrence (reading R0: the paper does not state the cell recurrence; the reading, its
boundary convention and its tie rule are listed in the design notes).

    forward(C, precision)  -> (D, sel)      precision in {"f64", "f32", "i64"}
    backward(sel, gD, gscore, precision) -> gC
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wf_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "tridiag.c"), os.path.join(_HERE, "softmin.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

SEL_NONE, SEL_NW, SEL_N, SEL_W = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, p = ctypes.c_int64, ctypes.c_void_p
    for name in ("wfo_forward_f64", "wfo_forward_f32", "wfo_forward_i64"):
        f = getattr(lib, name)
        f.argtypes = [i64, i64, p, i64, p, i64, p]
        f.restype = None
    lib.wfo_backward_f64.argtypes = [i64, i64, p, p, i64, ctypes.c_double, p, i64]
    lib.wfo_backward_f64.restype = None
    lib.wfo_backward_f32.argtypes = [i64, i64, p, p, i64, ctypes.c_float, p, i64]
    lib.wfo_backward_f32.restype = None
    lib.wfo_version.restype = ctypes.c_int
    i32 = ctypes.c_int32
    for suf in ("f64", "f32"):
        f = getattr(lib, "tro_thomas_" + suf)
        f.argtypes = [i64, p, p, p, p, p]
        f.restype = ctypes.c_int
        f = getattr(lib, "tro_interface_" + suf)
        f.argtypes = [i64, i64, p, p, p, p, p, p, p, p]
        f.restype = None
        f = getattr(lib, "tro_back_solve_" + suf)
        f.argtypes = [i64, i64, p, p, p, p, p, p]
        f.restype = ctypes.c_int
        f = getattr(lib, "tro_partition_" + suf)
        f.argtypes = [i64, i32, p, p, p, p, p, p]
        f.restype = ctypes.c_int
    d = ctypes.c_double
    lib.wfo_soft_forward_f64.argtypes = [i64, i64, p, i64, d, p, i64]
    lib.wfo_soft_forward_f64.restype = None
    lib.wfo_soft_backward_f64.argtypes = [i64, i64, p, i64, p, i64, d, p, i64, d, p, i64]
    lib.wfo_soft_backward_f64.restype = None
    lib.tro_subsystems.argtypes = [i64, i64]
    lib.tro_subsystems.restype = i64
    if lib.wfo_version() != 2:
        raise RuntimeError("stale oracle build")
    _lib = lib
    return lib


_FWD = {"f64": ("wfo_forward_f64", np.float64),
        "f32": ("wfo_forward_f32", np.float32),
        "i64": ("wfo_forward_i64", np.int64)}


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def forward(C, precision: str = "f64", want_sel: bool = True):
    """Row-by-row forward sweep.  Returns (D, sel); sel is None when want_sel is False.

    C is converted to the precision's type first (float32 data widens exactly to float64;
    integer data must fit int64)."""
    lib = _load()
    name, dt = _FWD[precision]
    C = np.ascontiguousarray(np.asarray(C), dtype=dt)
    if C.ndim != 2:
        raise ValueError("C must be 2-D")
    m, n = C.shape
    D = np.empty((m, n), dtype=dt)
    sel = np.empty((m, n), dtype=np.uint8) if want_sel else None
    if m and n:
        getattr(lib, name)(m, n, _ptr(C), n, _ptr(D), n, _ptr(sel) if want_sel else None)
    return D, sel


def score(C, precision: str = "f64"):
    D, _ = forward(C, precision, want_sel=False)
    return D[-1, -1]


def backward(sel, gD=None, gscore=0.0, precision: str = "f64"):
    """Routed adjoint for a fixed selection map; returns gC with the precision's type."""
    lib = _load()
    sel = np.ascontiguousarray(sel, dtype=np.uint8)
    m, n = sel.shape
    if precision == "f64":
        dt, fn = np.float64, lib.wfo_backward_f64
    elif precision == "f32":
        dt, fn = np.float32, lib.wfo_backward_f32
    else:
        raise ValueError(precision)
    gC = np.empty((m, n), dtype=dt)
    g = None
    if gD is not None:
        g = np.ascontiguousarray(gD, dtype=dt)
        assert g.shape == (m, n)
    if m and n:
        fn(m, n, _ptr(sel), _ptr(g) if g is not None else None, n, dt(gscore), _ptr(gC), n)
    return gC


def grad(C, gD=None, gscore=1.0, precision: str = "f64"):
    """Convenience: forward for SEL, then the adjoint."""
    D, sel = forward(C, precision if precision != "i64" else "f64")
    return backward(sel, gD, gscore, precision), D


# ------------------------------------------------------------------------------------------
# Smooth variant (softmin.c): the minimum of the three neighbours replaced by the soft minimum
# of temperature gamma; float64 only.

def soft_forward(C, gamma: float) -> np.ndarray:
    """D of the soft-min recurrence (float64; C must be finite)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    if C.ndim != 2 or C.size == 0:
        raise ValueError("C must be a non-empty 2-D array")
    if not gamma > 0:
        raise ValueError("gamma must be positive")
    m, n = C.shape
    D = np.empty_like(C)
    _load().wfo_soft_forward_f64(m, n, _ptr(C), n, float(gamma), _ptr(D), n)
    return D


def soft_backward(C, D, gamma: float, gD=None, gscore: float = 0.0) -> np.ndarray:
    """gC of L = sum(gD * D) + gscore * D[-1, -1] for the soft-min recurrence (float64)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    m, n = C.shape
    if D.shape != (m, n):
        raise ValueError("D must match C")
    g = None if gD is None else np.ascontiguousarray(gD, dtype=np.float64)
    gC = np.empty_like(C)
    _load().wfo_soft_backward_f64(m, n, _ptr(C), n, _ptr(D), n, float(gamma), _ptr(g) if g is not None else None,
                                  n, float(gscore), _ptr(gC), n)
    return gC
