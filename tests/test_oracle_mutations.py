"""The oracle's pins must catch plausible mistakes (CPU only).

Each case plants one mistake in a private copy of the oracle source (a dropped
predecessor, a wrong index, a transposed operand, a wrong tie rule, a dropped adjoint term),
builds it into a temporary library and checks that the brute-force / tie-rule / adjoint pins
reject it.  The shipped oracle is never modified.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from test_oracle_pins import brute_min

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "wf_oracle.c")

MUTATIONS = {
    "drop_nw": ("nw = (i > 0 && j > 0) ? D[(i - 1) * ldd + (j - 1)] : INF;", "nw = INF;"),
    "wrong_n_index": ("no = (i > 0) ? D[(i - 1) * ldd + j] : INF;",
                      "no = (i > 0) ? D[(i - 1) * ldd + (j > 0 ? j - 1 : j)] : INF;"),
    "transposed_c": ("D[i * ldd + j] = C[i * ldc + j] + v;", "D[i * ldd + j] = C[j * ldc + i] + v;"),
    "tie_rule": ("if (no < v) { v = no; s = WFO_SEL_N; }", "if (no <= v) { v = no; s = WFO_SEL_N; }"),
    "corner": ("nw = (T)0; no = INF; w = INF;", "nw = (T)1; no = INF; w = INF;"),
    "adjoint_drop_nw": ("a = a + gC[(i + 1) * ldgc + (j + 1)];", "a = a;"),
    "adjoint_wrong_sel": ("sel[i * n + (j + 1)] == WFO_SEL_W", "sel[i * n + (j + 1)] == WFO_SEL_N"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), str(c), "-lm"],
                   check=True)
    lib = ctypes.CDLL(str(so))
    i64, p = ctypes.c_int64, ctypes.c_void_p
    lib.wfo_forward_f64.argtypes = [i64, i64, p, i64, p, i64, p]
    lib.wfo_backward_f64.argtypes = [i64, i64, p, p, i64, ctypes.c_double, p, i64]
    return lib


def _fwd(lib, C):
    C = np.ascontiguousarray(C, dtype=np.float64)
    m, n = C.shape
    D = np.empty_like(C)
    sel = np.empty((m, n), dtype=np.uint8)
    lib.wfo_forward_f64(m, n, C.ctypes.data, n, D.ctypes.data, n, sel.ctypes.data)
    return D, sel


def _bwd(lib, sel, g):
    m, n = sel.shape
    gC = np.empty((m, n))
    lib.wfo_backward_f64(m, n, sel.ctypes.data, None, n, g, gC.ctypes.data, n)
    return gC


def _pins_pass(lib):
    rng = np.random.default_rng(0)
    for _ in range(6):
        k = int(rng.integers(2, 5))
        C = rng.integers(-3, 8, size=(k, k))
        D, sel = _fwd(lib, C)
        for i in range(k):
            for j in range(k):
                if D[i, j] != brute_min(C, i, j)[0]:
                    return False
        best, paths = brute_min(C, k - 1, k - 1)
        gC = _bwd(lib, sel, 1.0)
        if (gC * C).sum() != best:
            return False
        if len(paths) == 1:
            ref = np.zeros((k, k))
            for a, b in paths[0]:
                ref[a, b] = 1
            if not np.array_equal(ref, gC):
                return False
    # tie rule: all-zero interior ties go to NW, N beats W
    _, sel = _fwd(lib, np.zeros((3, 3)))
    if sel[1, 1] != 1:
        return False
    _, sel = _fwd(lib, np.array([[5.0, -1.0], [-1.0, 0.0]]))
    return sel[1, 1] == 2


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_unmutated_copy_passes(tmp_path):
    lib = _build(tmp_path, "identity", "enum { WFO_SEL_NONE = 0", "enum { WFO_SEL_NONE = 0")
    assert _pins_pass(lib)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    lib = _build(tmp_path, name, old, new)
    assert not _pins_pass(lib), f"pins did not catch mutation {name}"
