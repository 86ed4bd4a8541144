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
    "k without ckpt": dict(ckpt=None, ckpt_k=64),
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
