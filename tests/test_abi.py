"""The C ABI library loads, exports what include/wf.h declares, and validates arguments
before touching the device (CPU only: no call here reaches a HIP runtime function)."""
import ctypes

import pytest

from paper_2510_27351_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _lib.declared_symbols()
    assert {"wf_forward", "wf_last_async_error", "wf_error_string"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_error_strings(lib):
    assert _lib.error_string(0) == "ok"
    assert "argument" in _lib.error_string(_lib.WF_E_ARG)
    assert _lib.error_string(12345) == "unknown error"
    assert lib.wf_version() >= 100


def test_ckpt_elems(lib):
    # rows every 64 (all bands but the last) + block columns (all blocks but the last)
    assert lib.wf_ckpt_elems(2048, 2048, 64) == 31 * 2048 + 31 * 2048
    assert lib.wf_ckpt_elems(100, 50, 0) == 0
    assert lib.wf_ckpt_elems(64, 64, 64) == 0
    assert lib.wf_ckpt_elems(65, 130, 64) == 1 * 130 + 2 * 65
    assert lib.wf_ckpt_elems(0, 5, 64) == -1
    assert lib.wf_ckpt_elems(5, 5, -1) == -1


def test_set_tile_validation(lib):
    for t in (16, 32, 64, 0):
        assert lib.wf_set_tile(t) == 0
    for t in (1, 8, 128, -16):
        assert lib.wf_set_tile(t) == _lib.WF_E_ARG


BAD_FORWARD = {
    "bad dtype": dict(dtype=7),
    "m = 0": dict(m=0),
    "n = 0": dict(n=0),
    "negative n": dict(n=-3),
    "ldc < n": dict(ldc=3),
    "ldd < n": dict(ldd=3),
    "null C": dict(C=None),
    "null score": dict(score=None),
    "ckpt without k": dict(ckpt=0x1000, ckpt_k=0),
    "k without ckpt": dict(m=100, ckpt=None, ckpt_k=64),
    "k too large": dict(ckpt=0x1000, ckpt_k=5000),
    "m*n overflow": dict(m=1 << 40, n=1 << 31, ldc=1 << 31, ldd=1 << 31),
}


@pytest.mark.parametrize("case", sorted(BAD_FORWARD))
def test_forward_rejects_bad_arguments_before_device_work(lib, case):
    args = dict(dtype=0, m=8, n=8, C=0x1000, ldc=8, D=0x2000, ldd=8, score=0x3000, ckpt=None, ckpt_k=0,
                stream=None)
    args.update(BAD_FORWARD[case])
    rc = lib.wf_forward(args["dtype"], args["m"], args["n"], args["C"], args["ldc"], args["D"], args["ldd"],
                        args["score"], args["ckpt"], args["ckpt_k"], args["stream"])
    assert rc == _lib.WF_E_ARG, case


BAD_BACKWARD = {
    "bad dtype": dict(dtype=7),
    "int32 unsupported": dict(dtype=2, expect=_lib.WF_E_UNSUPPORTED),
    "m = 0": dict(m=0),
    "n = 0": dict(n=0),
    "ldc < n": dict(ldc=3),
    "ldgc < n": dict(ldgc=3),
    "ldgd < n": dict(ldgd=3),
    "ldd < n": dict(ldd=3),
    "null C": dict(C=None),
    "null g_C": dict(g_C=None),
    "neither D nor ckpt": dict(D=None),
    "both D and ckpt": dict(ckpt=0x5000, ckpt_k=64),
    "ckpt without k": dict(D=None, ckpt=0x5000, ckpt_k=0),
    "k without ckpt": dict(m=100, D=None, ckpt=None, ckpt_k=64),
    "k too large": dict(D=None, ckpt=0x5000, ckpt_k=5000),
    "m*n overflow": dict(m=1 << 40, n=1 << 31, ldc=1 << 31, ldd=1 << 31, ldgd=1 << 31, ldgc=1 << 31),
}


@pytest.mark.parametrize("case", sorted(BAD_BACKWARD))
def test_backward_rejects_bad_arguments_before_device_work(lib, case):
    args = dict(dtype=0, m=8, n=8, C=0x1000, ldc=8, ckpt=None, ckpt_k=0, D=0x2000, ldd=8, g_score=0x3000,
                g_D=0x4000, ldgd=8, g_C=0x6000, ldgc=8, stream=None, expect=_lib.WF_E_ARG)
    args.update(BAD_BACKWARD[case])
    rc = lib.wf_backward(args["dtype"], args["m"], args["n"], args["C"], args["ldc"], args["ckpt"], args["ckpt_k"],
                         args["D"], args["ldd"], args["g_score"], args["g_D"], args["ldgd"], args["g_C"],
                         args["ldgc"], args["stream"])
    assert rc == args["expect"], case


BAD_SELECT = {
    "bad dtype": dict(dtype=7),
    "int32 unsupported": dict(dtype=2, expect=_lib.WF_E_UNSUPPORTED),
    "m = 0": dict(m=0),
    "n = 0": dict(n=0),
    "ldc < n": dict(ldc=3),
    "null C": dict(C=None),
    "neither D nor ckpt": dict(D=None),
    "both D and ckpt": dict(ckpt=0x5000, ckpt_k=64),
    "k too large": dict(D=None, ckpt=0x5000, ckpt_k=5000),
}


@pytest.mark.parametrize("case", sorted(BAD_SELECT))
def test_select_rejects_bad_arguments_before_device_work(lib, case):
    args = dict(dtype=0, m=8, n=8, C=0x1000, ldc=8, ckpt=None, ckpt_k=0, D=0x2000, ldd=8, stream=None,
                expect=_lib.WF_E_ARG)
    args.update(BAD_SELECT[case])
    rc = lib.wf_select(args["dtype"], args["m"], args["n"], args["C"], args["ldc"], args["ckpt"], args["ckpt_k"],
                       args["D"], args["ldd"], args["stream"])
    assert rc == args["expect"], case


BAD_REVERSE = {
    "bad dtype": dict(dtype=7),
    "int32 unsupported": dict(dtype=2, expect=_lib.WF_E_UNSUPPORTED),
    "m = 0": dict(m=0),
    "n = 0": dict(n=0),
    "null g_C": dict(g_C=None),
    "ldgc < n": dict(ldgc=3),
    "ldgd < n": dict(ldgd=3),
    "m*n overflow": dict(m=1 << 40, n=1 << 31, ldgd=1 << 31, ldgc=1 << 31),
}


@pytest.mark.parametrize("case", sorted(BAD_REVERSE))
def test_reverse_rejects_bad_arguments_before_device_work(lib, case):
    args = dict(dtype=0, m=8, n=8, g_score=0x3000, g_D=0x4000, ldgd=8, g_C=0x6000, ldgc=8, stream=None,
                expect=_lib.WF_E_ARG)
    args.update(BAD_REVERSE[case])
    rc = lib.wf_reverse(args["dtype"], args["m"], args["n"], args["g_score"], args["g_D"], args["ldgd"],
                        args["g_C"], args["ldgc"], args["stream"])
    assert rc == args["expect"], case


# ------------------------------------------------------------------------------------------
# The tridiagonal solver's entry points (include/tri.h): exported, and argument errors are
# refused before any device work.

def test_every_tri_symbol_is_exported(lib):
    names = _lib.declared_symbols(_lib.TRI_HEADER)
    assert {"tri_stage1", "tri_stage3", "tri_thomas", "tri_solve", "tri_plan_create", "tri_predict"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_tri_subsystems_matches_the_oracle_partition(lib):
    from oracle import tridiag
    for N in (2, 3, 4, 5, 9, 10, 11, 100, 101, 4097):
        for m in (2, 3, 4, 7, 32, 64, 5000):
            assert lib.tri_subsystems(N, m) == len(tridiag.partition_sizes(N, m)), (N, m)
    assert lib.tri_subsystems(1, 4) == -1
    assert lib.tri_subsystems(10, 1) == -1


P = 0x1000  # a non-null pointer that no accepted call would reach


@pytest.mark.parametrize("args", [
    (7, 1, 100, 4),      # dtype
    (1, 0, 100, 4),      # batch
    (1, 1, 1, 4),        # N < 2
    (1, 1, 100, 1),      # m < 2
    (0, 1, 100, 1),
])
def test_tri_stage_argument_errors(lib, args):
    dt, batch, N, m = args
    assert lib.tri_stage1(dt, batch, N, m, P, P, P, P, P, P, P, P, None) == _lib.WF_E_ARG
    assert lib.tri_stage3(dt, batch, N, m, P, P, P, P, P, P, None) == _lib.WF_E_ARG


def test_tri_null_pointers_and_limits(lib):
    assert lib.tri_stage1(1, 1, 100, 4, None, P, P, P, P, P, P, P, None) == _lib.WF_E_ARG
    assert lib.tri_stage1(1, 1, 100, 4, P, P, P, P, P, P, P, None, None) == _lib.WF_E_ARG
    assert lib.tri_stage3(1, 1, 100, 4, P, P, P, P, None, P, None) == _lib.WF_E_ARG
    assert lib.tri_thomas(1, 1, 100, P, P, P, P, P, None, None) == _lib.WF_E_ARG
    assert lib.tri_thomas(1, 1, 0, P, P, P, P, P, P, None) == _lib.WF_E_ARG
    # a sub-system must fit in one workgroup's LDS
    assert lib.tri_stage1(1, 1, 100000, 5000, P, P, P, P, P, P, P, P, None) == _lib.WF_E_UNSUPPORTED
    assert lib.tri_stage1(0, 1, 100000, 9000, P, P, P, P, P, P, P, P, None) == _lib.WF_E_UNSUPPORTED
    assert lib.tri_solve(None, P, P, P, P, P, None) == _lib.WF_E_ARG


def test_tri_plan_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.tri_plan_create(None, 1, 1, 100, 4, 0, None) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 7, 1, 100, 4, 0, None) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 1, 0, 100, 4, 0, None) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 1, 1, 0, 4, 0, None) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 1, 1, 100, 1, 0, None) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 1, 1, 100, 4, 7, None) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 1, 1, 100, 4, -2, None) == _lib.WF_E_ARG
    bad = (ctypes.c_int32 * 2)(10, 1)
    assert lib.tri_plan_create(ctypes.byref(h), 1, 1, 100000, 4, 2, bad) == _lib.WF_E_ARG
    assert lib.tri_plan_create(ctypes.byref(h), 1, 1, 100000, 3000, 0, None) == _lib.WF_E_UNSUPPORTED
    assert not h.value


def test_tri_predict_validation(lib):
    m, R = ctypes.c_int32(), ctypes.c_int32()
    assert lib.tri_predict(7, 1000, ctypes.byref(m), ctypes.byref(R), None) == _lib.WF_E_ARG
    assert lib.tri_predict(1, 0, ctypes.byref(m), ctypes.byref(R), None) == _lib.WF_E_ARG
    assert lib.tri_predict(1, 1000, ctypes.byref(m), ctypes.byref(R), None) == 0
    assert m.value >= 2 and 0 <= R.value <= 6
