"""ctypes binding of libwf.so (include/wf.h, include/tri.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "wf.h")
TRI_HEADER = os.path.join(os.path.dirname(HERE), "include", "tri.h")

WF_F32, WF_F64, WF_I32 = 0, 1, 2
WF_OK, WF_E_ARG, WF_E_UNSUPPORTED, WF_E_NOMEM, WF_E_DEVICE, WF_E_TIMEOUT = range(6)

_lib = None


class WfError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {error_string(code)} (code {code})")


def load():
    """Loads libwf.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libwf.so is not built ({LIB_PATH}); run python -m paper_2510_27351_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.wf_forward.argtypes = [ctypes.c_int, i64, i64, p, i64, p, i64, p, p, i32, p]
    lib.wf_forward.restype = ctypes.c_int
    lib.wf_backward.argtypes = [ctypes.c_int, i64, i64, p, i64, p, i32, p, i64, p, p, i64, p, i64, p]
    lib.wf_backward.restype = ctypes.c_int
    lib.wf_select.argtypes = [ctypes.c_int, i64, i64, p, i64, p, i32, p, i64, p]
    lib.wf_select.restype = ctypes.c_int
    lib.wf_reverse.argtypes = [ctypes.c_int, i64, i64, p, p, i64, p, i64, p]
    lib.wf_reverse.restype = ctypes.c_int
    pi64 = ctypes.POINTER(i64)
    lib.wf_plan_create.argtypes = [ctypes.POINTER(p), ctypes.c_int, i32, pi64, pi64, pi64, i32, i32, p]
    lib.wf_plan_create.restype = ctypes.c_int
    lib.wf_plan_elems.argtypes = [p]
    lib.wf_plan_elems.restype = i64
    lib.wf_plan_offsets.argtypes = [p, pi64]
    lib.wf_plan_offsets.restype = ctypes.c_int
    lib.wf_plan_config.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.wf_plan_config.restype = ctypes.c_int
    lib.wf_batch_forward.argtypes = [p, p, p, p, p]
    lib.wf_batch_forward.restype = ctypes.c_int
    lib.wf_plan_ckpt_elems.argtypes = [p, i32]
    lib.wf_plan_ckpt_elems.restype = i64
    lib.wf_plan_ckpt_offsets.argtypes = [p, i32, pi64]
    lib.wf_plan_ckpt_offsets.restype = ctypes.c_int
    lib.wf_batch_forward_ckpt.argtypes = [p, p, p, p, p, i32, p]
    lib.wf_batch_forward_ckpt.restype = ctypes.c_int
    lib.wf_batch_backward.argtypes = [p, p, p, i32, p, p, p, p, p]
    lib.wf_batch_backward.restype = ctypes.c_int
    lib.wf_plan_destroy.argtypes = [p]
    lib.wf_plan_destroy.restype = None
    lib.wf_forward_noalloc.argtypes = [ctypes.c_int, i64, i64, p, i64, p, i64, p, p, i32, p]
    lib.wf_forward_noalloc.restype = ctypes.c_int
    dbl = ctypes.c_double
    lib.wf_soft_forward.argtypes = [ctypes.c_int, i64, i64, dbl, p, i64, p, i64, p, p]
    lib.wf_soft_forward.restype = ctypes.c_int
    lib.wf_soft_backward.argtypes = [ctypes.c_int, i64, i64, dbl, p, i64, p, i64, p, p, i64, p, i64, p]
    lib.wf_soft_backward.restype = ctypes.c_int
    lib.wf_ckpt_elems.argtypes = [i64, i64, i32]
    lib.wf_ckpt_elems.restype = i64
    lib.wf_set_tile.argtypes = [i32]
    lib.wf_set_tile.restype = ctypes.c_int
    lib.wf_tile_predict.argtypes = [i32, i64, i64, i32]
    lib.wf_tile_predict.restype = i32
    lib.wf_last_async_error.argtypes = [p]
    lib.wf_last_async_error.restype = ctypes.c_int
    lib.wf_error_string.argtypes = [ctypes.c_int]
    lib.wf_error_string.restype = ctypes.c_char_p
    lib.wf_trace_enable.argtypes = [i64]
    lib.wf_trace_enable.restype = ctypes.c_int
    lib.wf_trace_fetch.argtypes = [p, i64]
    lib.wf_trace_fetch.restype = i64
    lib.wf_fault_inject.argtypes = [i32]
    lib.wf_fault_inject.restype = ctypes.c_int
    lib.wf_version.argtypes = []
    lib.wf_version.restype = ctypes.c_int
    # tridiagonal partition solver (include/tri.h)
    pi32 = ctypes.POINTER(i32)
    lib.tri_stage1.argtypes = [ctypes.c_int, i32, i64, i32, p, p, p, p, p, p, p, p, p]
    lib.tri_stage1.restype = ctypes.c_int
    lib.tri_stage3.argtypes = [ctypes.c_int, i32, i64, i32, p, p, p, p, p, p, p]
    lib.tri_stage3.restype = ctypes.c_int
    lib.tri_thomas.argtypes = [ctypes.c_int, i32, i64, p, p, p, p, p, p, p]
    lib.tri_thomas.restype = ctypes.c_int
    lib.tri_subsystems.argtypes = [i64, i32]
    lib.tri_subsystems.restype = i64
    lib.tri_plan_create.argtypes = [ctypes.POINTER(p), ctypes.c_int, i32, i64, i32, i32, pi32]
    lib.tri_plan_create.restype = ctypes.c_int
    lib.tri_plan_config.argtypes = [p, pi32, pi32, pi32, pi64]
    lib.tri_plan_config.restype = ctypes.c_int
    lib.tri_solve.argtypes = [p, p, p, p, p, p, p]
    lib.tri_solve.restype = ctypes.c_int
    lib.tri_plan_level.argtypes = [p, i32, p, p, p, p, p]
    lib.tri_plan_level.restype = ctypes.c_int
    lib.tri_plan_destroy.argtypes = [p]
    lib.tri_plan_destroy.restype = None
    lib.tri_predict.argtypes = [ctypes.c_int, i64, pi32, pi32, pi32]
    lib.tri_predict.restype = ctypes.c_int
    _lib = lib
    return lib


def error_string(code: int) -> str:
    return load().wf_error_string(code).decode()


def check(code: int, what: str) -> None:
    if code != WF_OK:
        raise WfError(code, what)


def declared_symbols(header: str = HEADER) -> list[str]:
    """Names of the functions declared in a header of include/ (wf.h by default)."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:wf|tri)_[a-z_0-9]+)\s*\(", text)))
