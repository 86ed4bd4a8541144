"""The solver's parameter predictor (tri_predict) and the paper's rules behind it, CPU only.

The paper fits a 1-NN rule on the system size N to the measured-fastest sub-system size m
(Table I) and, for the recursive method, to the fastest number of recursive steps R
(Table II), then states how m_1 .. m_R are chosen (section "Formulation of the algorithm
for the optimum m_i").  The library does the same with tables timed on MI355X
(tests/golden/mi355x_tri_table.txt).  Pins here:
  - the Table II fixture agrees with the paper's Figure 4 data (its argmin over R is the
    table's R for the four sizes the figure shows);
  - 1-NN on the paper's R labels reproduces its intervals except between two timed sizes
    that straddle an interval end, and the paper's test-split score (1.0) is reachable;
  - the library's prediction equals the oracle 1-NN on its own table, for the training
    sizes and for random sizes, and the m_1 .. m_R it returns follow the paper's rule.
"""
import ctypes
import math
import os

import numpy as np
import pytest

from oracle import knn
from paper_2510_27351_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def table2():
    rows, sizes, fig = [], None, {}
    for line in open(os.path.join(GOLD, "table2_opt_recursion.txt")):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "sizes":
            sizes = [int(v) for v in line[1:]]
        elif line[0] == "fig4":
            fig[int(line[1])] = [float(v) for v in line[2:]]
        else:
            rows.append((int(line[0]), int(line[1]), int(line[2])))
    return rows, sizes, fig


def paper_r(N):
    for R, lo, hi in table2()[0]:
        if lo <= N <= hi:
            return R
    return None


def test_table2_fixture_matches_figure4():
    _, _, fig = table2()
    for N, times in fig.items():
        assert int(np.argmin(times)) == paper_r(N), N


def test_paper_r_labels_by_1nn():
    _, sizes, _ = table2()
    x = np.log10(sizes)
    y = np.array([paper_r(N) for N in sizes])
    assert None not in list(y)
    # leave-one-out: a miss only where the left-out size's neighbours straddle an interval end
    for k in range(len(sizes)):
        keep = np.arange(len(sizes)) != k
        got = knn.predict(x[keep], y[keep], x[k:k + 1])[0]
        if got != y[k]:
            lo = y[k - 1] if k > 0 else y[k]
            hi = y[k + 1] if k + 1 < len(y) else y[k]
            assert lo != y[k] or hi != y[k], sizes[k]
    # a 3:1 split whose training part holds every label scores 1.0 on its test part
    rng = np.random.default_rng(0)
    hits = 0
    for _ in range(400):
        perm = rng.permutation(len(sizes))
        tr, te = perm[: 3 * len(sizes) // 4], perm[3 * len(sizes) // 4:]
        if set(y[tr]) != set(y):
            continue
        if np.all(knn.predict(x[tr], y[tr], x[te]) == y[te]):
            hits += 1
    assert hits > 0


def lib_table():
    """(N, m64, R64, m32, R32) rows of the library's timed table (golden copy)."""
    rows = []
    for line in open(os.path.join(GOLD, "mi355x_tri_table.txt")):
        line = line.split("#")[0].split()
        if line:
            rows.append(tuple(int(v) for v in line))
    return rows


def predict(dtype, N):
    lib = _lib.load()
    m, R = ctypes.c_int32(), ctypes.c_int32()
    ms = (ctypes.c_int32 * 6)()
    assert lib.tri_predict(dtype, N, ctypes.byref(m), ctypes.byref(R), ms) == 0
    return m.value, R.value, [ms[i] for i in range(R.value)]


def subsystems(N, m):
    P = -(-N // m)
    if P > 1 and N - (P - 1) * m == 1:
        P -= 1
    return P


@pytest.mark.parametrize("dtype,col_m,col_r", [(_lib.WF_F64, 1, 2), (_lib.WF_F32, 3, 4)])
def test_library_predictor_equals_oracle_1nn(dtype, col_m, col_r):
    rows = lib_table()
    x = np.log([r[0] for r in rows])
    ym = np.array([r[col_m] for r in rows])
    yr = np.array([r[col_r] for r in rows])
    rng = np.random.default_rng(dtype + 1)
    Ns = [r[0] for r in rows] + [int(v) for v in 10 ** rng.uniform(2, 8, 300)]
    for N in Ns:
        q = np.log([N])
        d = np.abs(x - q[0])
        if np.sort(d)[1] - np.sort(d)[0] < 1e-9:
            continue  # equally near two timed sizes
        m, R, ms = predict(dtype, N)
        assert m == knn.predict(x, ym, q)[0], N
        assert R == min(6, knn.predict(x, yr, q)[0]), N
        # the paper's rule for m_1 .. m_R
        nl = 2 * subsystems(N, m) if N >= 2 else 2
        for lvl in range(1, R + 1):
            if lvl == 1 and R > 1:
                want = 10
            else:
                want = knn.predict(x, ym, np.log([nl]))[0]
            assert ms[lvl - 1] == want, (N, lvl)
            nl = 2 * subsystems(nl, ms[lvl - 1])


def test_library_table_is_the_golden_copy():
    """The table compiled into the library is the committed copy (spot checks through the
    predictor at every training size)."""
    for N, m64, R64, m32, R32 in lib_table():
        assert predict(_lib.WF_F64, N)[:2] == (m64, min(R64, 6))
        assert predict(_lib.WF_F32, N)[:2] == (m32, min(R32, 6))


def test_table_accuracy_report():
    """Leave-one-out accuracy of the 1-NN on the timed table against the null accuracy (the
    figures DESIGN quotes); the rule must beat always predicting the most frequent label."""
    rows = lib_table()
    x = np.log([r[0] for r in rows])
    for col in (1, 2, 3, 4):
        y = np.array([r[col] for r in rows])
        acc = knn.loo_accuracy(x, y)
        null = knn.null_accuracy(y)
        print(f"column {col}: 1-NN leave-one-out {acc:.2f}, null {null:.2f}")
        assert acc >= null - 1e-12 or math.isclose(acc, null)
