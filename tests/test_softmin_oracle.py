"""Pins of the soft-min oracle (oracle/softmin.c), CPU only.

What fixes the soft-min recurrence independently of its row-by-row code:
  - path enumeration: D[i][j] = -gamma log sum over all monotone (right, down, diagonal)
    paths from (0,0) to (i,j) of exp(-cost / gamma);
  - its gradient: dD[p][q]/dC[i][j] is the Gibbs probability (weights exp(-cost/gamma))
    that a path to (p,q) passes through (i,j);
  - the limit gamma -> 0: each soft minimum lies in [min - gamma log 3, min], so
    D_0 - (i+j) gamma log 3 <= D_gamma <= D_0 (D_0 from the min-plus oracle);
  - single rows and columns: prefix sums (one finite argument: the soft minimum is it);
  - central finite differences of the double forward;
and planted mistakes in a copy of the source are caught by these pins.
"""
import ctypes
import itertools
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "softmin.c")


def paths(i, j):
    """Every monotone path from (0,0) to (i,j) as a list of cells."""
    out = []

    def rec(p, q, acc):
        if (p, q) == (0, 0):
            out.append(list(reversed(acc + [(0, 0)])))
            return
        if p > 0 and q > 0:
            rec(p - 1, q - 1, acc + [(p, q)])
        if p > 0:
            rec(p - 1, q, acc + [(p, q)])
        if q > 0:
            rec(p, q - 1, acc + [(p, q)])

    rec(i, j, [])
    return out


def gibbs(C, i, j, gamma):
    """(-gamma log Z, the path list, their probabilities) over the paths to (i,j)."""
    ps = paths(i, j)
    costs = np.array([math.fsum(C[p][q] for p, q in path) for path in ps])
    lo = costs.min()
    w = np.exp(-(costs - lo) / gamma)
    Z = math.fsum(w)
    return lo - gamma * math.log(Z), ps, w / Z


def test_path_counts_are_delannoy():
    assert [len(paths(k, k)) for k in range(6)] == [1, 3, 13, 63, 321, 1683]


@pytest.mark.parametrize("gamma", [0.05, 0.5, 2.0])
@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (4, 1), (3, 3), (4, 5), (5, 4)])
def test_forward_equals_path_enumeration(shape, gamma):
    C = np.random.default_rng(shape[0] * 7 + shape[1]).uniform(-1, 2, shape)
    D = oracle.soft_forward(C, gamma)
    for i in range(shape[0]):
        for j in range(shape[1]):
            want = gibbs(C, i, j, gamma)[0]
            assert abs(D[i, j] - want) <= 1e-12 * max(1.0, abs(want)), (i, j)


@pytest.mark.parametrize("gamma", [0.1, 1.0])
def test_score_gradient_is_path_probability(gamma):
    C = np.random.default_rng(5).uniform(0, 1, (4, 5))
    D = oracle.soft_forward(C, gamma)
    g = oracle.soft_backward(C, D, gamma, gscore=1.0)
    _, ps, prob = gibbs(C, 3, 4, gamma)
    want = np.zeros_like(C)
    for path, pr in zip(ps, prob):
        for p, q in path:
            want[p, q] += pr
    assert np.max(np.abs(g - want)) <= 1e-12


def test_table_gradient_is_weighted_path_probability():
    """gD upstream: dL/dC[i][j] = sum_(p,q) gD[p][q] P(path to (p,q) passes (i,j))."""
    gamma = 0.3
    rng = np.random.default_rng(9)
    C = rng.uniform(0, 1, (3, 4))
    gD = rng.uniform(-1, 1, (3, 4))
    D = oracle.soft_forward(C, gamma)
    g = oracle.soft_backward(C, D, gamma, gD=gD, gscore=0.5)
    want = np.zeros_like(C)
    for p, q in itertools.product(range(3), range(4)):
        up = gD[p, q] + (0.5 if (p, q) == (2, 3) else 0.0)
        _, ps, prob = gibbs(C, p, q, gamma)
        for path, pr in zip(ps, prob):
            for i, j in path:
                want[i, j] += up * pr
    assert np.max(np.abs(g - want)) <= 1e-12


def test_small_gamma_is_bracketed_by_min_plus():
    C = np.random.default_rng(2).uniform(0, 1, (30, 40))
    D0, _ = oracle.forward(C, "f64", want_sel=False)
    for gamma in (0.001, 0.01, 0.1):
        D = oracle.soft_forward(C, gamma)
        i, j = np.indices(C.shape)
        assert np.all(D <= D0 + 1e-12)
        assert np.all(D >= D0 - (i + j) * gamma * math.log(3) - 1e-12)


def test_single_row_and_column_are_prefix_sums():
    C = np.random.default_rng(3).uniform(-1, 1, (1, 50))
    assert np.array_equal(oracle.soft_forward(C, 0.7)[0], np.cumsum(C[0]))
    assert np.array_equal(oracle.soft_forward(C.T, 0.7)[:, 0], np.cumsum(C[0]))


def test_central_differences():
    gamma, h = 0.25, 1e-5
    rng = np.random.default_rng(4)
    C = rng.uniform(0, 1, (12, 15))
    gD = rng.uniform(-1, 1, C.shape)

    def loss(Cx):
        D = oracle.soft_forward(Cx, gamma)
        return float((gD * D).sum() + 0.75 * D[-1, -1])

    g = oracle.soft_backward(C, oracle.soft_forward(C, gamma), gamma, gD=gD, gscore=0.75)
    for i, j in [(0, 0), (3, 7), (11, 14), (6, 0), (0, 9), (10, 2)]:
        Cp, Cm = C.copy(), C.copy()
        Cp[i, j] += h
        Cm[i, j] -= h
        fd = (loss(Cp) - loss(Cm)) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-7 * max(1.0, abs(g[i, j])), (i, j, fd, g[i, j])


# ------------------------------------------------------------------------------------------
# planted mistakes

MUTATIONS = {
    "drop_nw": ("x[0] = (i == 0 && j == 0) ? 0.0 : (i > 0 && j > 0) ? D[(i - 1) * ldd + (j - 1)] : INFINITY;",
                "x[0] = (i == 0 && j == 0) ? 0.0 : INFINITY;"),
    "sign_of_exponent": ("s += exp((mn - x[k]) / gamma);", "s += exp((x[k] - mn) / gamma);"),
    "gamma_dropped": ("(mn - gamma * log(s))", "(mn - log(s))"),
    "weight_without_c": ("e = e + exp((D[p * ldd + q] - C[p * ldc + q] - dij) / gamma) * gC[p * ldgc + q];\n      }\n      if (i + 1 < m) {",
                         "e = e + exp((D[p * ldd + q] - dij) / gamma) * gC[p * ldgc + q];\n      }\n      if (i + 1 < m) {"),
    "east_uses_south": ("const int64_t p = i, q = j + 1;", "const int64_t p = i + 1 < m ? i + 1 : i, q = j + 1;"),
    "corner": ("(i == 0 && j == 0) ? 0.0 :", "(i == 0 && j == 0) ? 1.0 :"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), str(c), "-lm"],
                   check=True)
    lib = ctypes.CDLL(str(so))
    i64, p, d = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    lib.wfo_soft_forward_f64.argtypes = [i64, i64, p, i64, d, p, i64]
    lib.wfo_soft_backward_f64.argtypes = [i64, i64, p, i64, p, i64, d, p, i64, d, p, i64]
    return lib


def _pins_pass(lib):
    gamma = 0.4
    C = np.ascontiguousarray(np.random.default_rng(1).uniform(0, 1, (3, 4)))
    D = np.empty_like(C)
    lib.wfo_soft_forward_f64(3, 4, C.ctypes.data, 4, gamma, D.ctypes.data, 4)
    for i in range(3):
        for j in range(4):
            if abs(D[i, j] - gibbs(C, i, j, gamma)[0]) > 1e-12:
                return False
    g = np.empty_like(C)
    lib.wfo_soft_backward_f64(3, 4, C.ctypes.data, 4, D.ctypes.data, 4, gamma, None, 4, 1.0, g.ctypes.data, 4)
    _, ps, prob = gibbs(C, 2, 3, gamma)
    want = np.zeros_like(C)
    for path, pr in zip(ps, prob):
        for p, q in path:
            want[p, q] += pr
    return bool(np.max(np.abs(g - want)) <= 1e-12)


def test_unmodified_copy_passes(tmp_path):
    lib = _build(tmp_path, "same", "gamma > 0", "gamma > 0")
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))
