"""Pins of the CPU oracle against things other than itself (CPU only).

The paper prints no worked example, table or value for the wavefront recurrence, so the
oracle is pinned by: exhaustive enumeration of monotone paths on tiny inputs (a different
algorithm: min over all paths instead of the recurrence), closed forms, invariants of the
min-plus recurrence, and properties of the routed adjoint (path structure, Euler identity
for a degree-1 positively homogeneous function, central finite differences).  Each pin is
chosen so that a dropped predecessor, a wrong index, a transposed operand or a wrong tie
rule fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

# ------------------------------------------------------------------ brute force helpers


def monotone_paths(i, j):
    """All paths from (0,0) to (i,j) using steps (0,1), (1,0), (1,1)."""
    if i == 0 and j == 0:
        yield [(0, 0)]
        return
    if j > 0:
        for p in monotone_paths(i, j - 1):
            yield p + [(i, j)]
    if i > 0:
        for p in monotone_paths(i - 1, j):
            yield p + [(i, j)]
    if i > 0 and j > 0:
        for p in monotone_paths(i - 1, j - 1):
            yield p + [(i, j)]


def brute_min(C, i, j):
    best, arg = None, []
    for p in monotone_paths(i, j):
        s = sum(int(C[a][b]) for a, b in p)
        if best is None or s < best:
            best, arg = s, [p]
        elif s == best:
            arg.append(p)
    return best, arg


def delannoy(a, b):
    return sum(math.comb(a, k) * math.comb(b, k) * 2 ** k for k in range(min(a, b) + 1))


# ------------------------------------------------------------------ forward pins


def test_path_enumerator_counts_are_delannoy():
    # the enumerator itself is checked against the closed-form path count
    for a in range(5):
        for b in range(5):
            assert sum(1 for _ in monotone_paths(a, b)) == delannoy(a, b)
    assert [delannoy(k, k) for k in range(7)] == [1, 3, 13, 63, 321, 1683, 8989]


@pytest.mark.parametrize("seed", range(12))
def test_forward_equals_min_over_all_paths(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    m, n = rng.integers(1, 6, size=2)
    C = rng.integers(-5, 10, size=(m, n))
    D64, _ = oracle_mod.forward(C.astype(np.float64), "f64")
    D32, _ = oracle_mod.forward(C.astype(np.float32), "f32")
    Di, _ = oracle_mod.forward(C, "i64")
    for i in range(m):
        for j in range(n):
            best, _ = brute_min(C, i, j)
            assert D64[i, j] == best
            assert D32[i, j] == best
            assert Di[i, j] == best


def test_hand_worked_example(oracle_mod):
    # Worked by hand from the recurrence (virtual row/column +inf, corner 0):
    #   C = 1 3 1      row 0 is a prefix sum: 1 4 5; column 0: 1 2 6
    #       1 5 1      D11 = 5 + min(1,4,2) = 6   D12 = 1 + min(4,5,6) = 5
    #       4 2 1      D21 = 2 + min(2,6,6) = 4   D22 = 1 + min(6,5,4) = 5
    # the argmin path is (0,0) -> (1,0) -> (2,1) -> (2,2), of cost 1+1+2+1 = 5.
    C = np.array([[1, 3, 1], [1, 5, 1], [4, 2, 1]], dtype=np.float64)
    D, sel = oracle_mod.forward(C)
    assert D.tolist() == [[1, 4, 5], [2, 6, 5], [6, 4, 5]]
    assert sel[2, 2] == oracle_mod.SEL_W and sel[2, 1] == oracle_mod.SEL_NW
    assert sel[1, 0] == oracle_mod.SEL_N and sel[0, 0] == oracle_mod.SEL_NONE
    gC = oracle_mod.backward(sel, None, 1.0)
    assert gC.tolist() == [[1, 0, 0], [1, 0, 0], [0, 1, 1]]


def test_constant_input_closed_form(oracle_mod):
    for c in (0.0, 0.5, 3.0):
        C = np.full((9, 13), c)
        D, _ = oracle_mod.forward(C)
        i, j = np.indices(C.shape)
        assert np.array_equal(D, c * (np.maximum(i, j) + 1))


def test_single_row_and_column_are_prefix_sums(oracle_mod):
    rng = np.random.default_rng(3)
    x = rng.random(257).astype(np.float32)
    D, _ = oracle_mod.forward(x[None, :], "f32")
    ref = np.empty_like(x)
    acc = np.float32(0)
    for k, v in enumerate(x):  # sequential single-precision sum, one rounding per step
        acc = np.float32(acc + v)
        ref[k] = acc
    assert np.array_equal(D[0], ref)
    Dt, _ = oracle_mod.forward(x[:, None], "f32")
    assert np.array_equal(Dt[:, 0], ref)


def test_zero_diagonal_gives_zero(oracle_mod):
    rng = np.random.default_rng(4)
    C = rng.random((20, 20)) + 0.25
    np.fill_diagonal(C, 0.0)
    D, _ = oracle_mod.forward(C)
    assert np.all(np.diag(D) == 0.0)
    assert np.all(D >= 0.0)


def test_dtw_of_identical_sequences_is_zero(oracle_mod):
    rng = np.random.default_rng(5)
    x = rng.random(31)
    C = np.abs(x[:, None] - x[None, :])
    assert oracle_mod.score(C) == 0.0
    # and of a time-stretched copy: repeating samples costs nothing
    y = np.repeat(x, 2)
    C2 = np.abs(x[:, None] - y[None, :])
    assert oracle_mod.score(C2) == 0.0


# ------------------------------------------------------------------ invariants


def test_power_of_two_scaling_is_bit_exact(oracle_mod):
    rng = np.random.default_rng(6)
    C = rng.standard_normal((40, 33)).astype(np.float32)
    D, _ = oracle_mod.forward(C, "f32")
    for k in (-3, 1, 7):
        Dk, _ = oracle_mod.forward(C * np.float32(2.0 ** k), "f32")
        assert np.array_equal(Dk, D * np.float32(2.0 ** k))


def test_transpose_symmetry(oracle_mod):
    rng = np.random.default_rng(7)
    C = rng.random((23, 37))
    D, _ = oracle_mod.forward(C)
    Dt, _ = oracle_mod.forward(C.T.copy())
    assert np.array_equal(Dt, D.T)


def test_monotone_and_lipschitz(oracle_mod):
    rng = np.random.default_rng(8)
    C = rng.standard_normal((30, 25))
    dC = rng.random((30, 25)) * 1e-3
    D, _ = oracle_mod.forward(C)
    D2, _ = oracle_mod.forward(C + dC)
    assert np.all(D2 >= D)
    m, n = C.shape
    assert np.max(np.abs(D2 - D)) <= (m + n - 1) * np.max(np.abs(dC)) * (1 + 1e-12)


def test_anti_diagonal_order_matches_row_order(oracle_mod):
    # evaluating the same recurrence one anti-diagonal at a time (a different schedule)
    rng = np.random.default_rng(9)
    m, n = 17, 29
    C = rng.random((m, n)).astype(np.float32)
    D, _ = oracle_mod.forward(C, "f32")
    inf = np.float32(np.inf)
    P = np.full((m + 1, n + 1), inf, dtype=np.float32)
    P[0, 0] = 0
    for d in range(m + n - 1):
        i = np.arange(max(0, d - n + 1), min(m, d + 1))
        j = d - i
        v = np.minimum(np.minimum(P[i, j], P[i, j + 1]), P[i + 1, j])
        P[i + 1, j + 1] = C[i, j] + v
    assert np.array_equal(P[1:, 1:], D)


def test_f32_within_rounding_bound_of_f64(oracle_mod):
    rng = np.random.default_rng(10)
    C = rng.random((200, 300)).astype(np.float32)
    D32, _ = oracle_mod.forward(C, "f32")
    D64, _ = oracle_mod.forward(C, "f64")
    i, j = np.indices(C.shape)
    u = 2.0 ** -24
    # positive terms: a path sum of k <= i+j+1 terms carries relative error <= (k-1) u / (1-(k-1)u)
    bound = (i + j) * u / (1 - (i + j) * u) * D64
    assert np.all(np.abs(D32.astype(np.float64) - D64) <= bound)


def test_integer_and_float_forms_agree_on_integers(oracle_mod):
    rng = np.random.default_rng(11)
    C = rng.integers(0, 1000, size=(64, 80))
    Di, si = oracle_mod.forward(C, "i64")
    Df, sf = oracle_mod.forward(C.astype(np.float64), "f64")
    assert np.array_equal(Di, Df.astype(np.int64))
    assert np.array_equal(si, sf)


def test_tie_rule_prefers_nw_then_n(oracle_mod):
    C = np.zeros((3, 3))
    _, sel = oracle_mod.forward(C)
    # all predecessors tie at 0 in the interior: NW wins
    assert sel[1, 1] == oracle_mod.SEL_NW and sel[2, 2] == oracle_mod.SEL_NW
    # first row / column: only one finite predecessor
    assert sel[0, 1] == oracle_mod.SEL_W and sel[1, 0] == oracle_mod.SEL_N
    # N beats W on a tie when NW is larger
    C = np.array([[5.0, -1.0], [-1.0, 0.0]])  # NW = 5, N = W = 4
    D, sel = oracle_mod.forward(C)
    assert D[1, 1] == 4.0 and sel[1, 1] == oracle_mod.SEL_N
    C = np.array([[5.0, -1.0], [-2.0, 0.0]])  # NW = 5, N = 4, W = 3
    _, sel = oracle_mod.forward(C)
    assert sel[1, 1] == oracle_mod.SEL_W


# ------------------------------------------------------------------ adjoint pins


def _is_monotone_path(mask):
    cells = sorted(zip(*np.nonzero(mask)))
    if not cells or cells[0] != (0, 0) or cells[-1] != (mask.shape[0] - 1, mask.shape[1] - 1):
        return False
    for (a, b), (c, d) in zip(cells, cells[1:]):
        if (c - a, d - b) not in ((0, 1), (1, 0), (1, 1)):
            return False
    return True


@pytest.mark.parametrize("seed", range(8))
def test_score_gradient_is_the_unique_argmin_path(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    m, n = rng.integers(1, 6, size=2)
    C = rng.integers(0, 50, size=(m, n))
    best, paths = brute_min(C, m - 1, n - 1)
    D, sel = oracle_mod.forward(C.astype(np.float64))
    gC = oracle_mod.backward(sel, None, 1.0)
    assert set(np.unique(gC)) <= {0.0, 1.0}
    assert _is_monotone_path(gC)
    assert (gC * C).sum() == best == D[-1, -1]
    if len(paths) == 1:
        ref = np.zeros((m, n))
        for a, b in paths[0]:
            ref[a, b] = 1
        assert np.array_equal(gC, ref)


@pytest.mark.parametrize("seed", range(6))
def test_table_gradient_matches_brute_force(oracle_mod, seed):
    # L = sum(gD * D): dL/dC = sum over cells of gD[cell] * (argmin path indicator of cell)
    rng = np.random.default_rng(200 + seed)
    m, n = rng.integers(2, 6, size=2)
    C = rng.permutation(m * n).reshape(m, n) * 7 + rng.integers(0, 3, size=(m, n))
    gD = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
    ref = np.zeros((m, n))
    unique = True
    for i in range(m):
        for j in range(n):
            _, paths = brute_min(C, i, j)
            unique &= len(paths) == 1
            for a, b in paths[0]:
                ref[a, b] += gD[i, j]
    D, sel = oracle_mod.forward(C.astype(np.float64))
    gC = oracle_mod.backward(sel, gD, 0.0)
    if unique:
        assert np.array_equal(gC, ref)


def test_euler_identity_and_linearity(oracle_mod):
    rng = np.random.default_rng(12)
    C = rng.random((40, 50))
    gD = rng.standard_normal((40, 50))
    D, sel = oracle_mod.forward(C)
    gC = oracle_mod.backward(sel, gD, 2.5)
    lhs = (C * gC).sum()
    rhs = (gD * D).sum() + 2.5 * D[-1, -1]
    assert abs(lhs - rhs) <= 1e-9 * (np.abs(C * gC).sum() + abs(rhs))
    g1 = oracle_mod.backward(sel, gD, 0.0)
    g2 = oracle_mod.backward(sel, None, 1.0)
    assert np.allclose(gC, g1 + 2.5 * g2, rtol=1e-12, atol=1e-12)


def test_central_finite_differences(oracle_mod):
    rng = np.random.default_rng(13)
    C = rng.random((24, 24))
    D, sel = oracle_mod.forward(C)
    gD = rng.standard_normal((24, 24))
    gC = oracle_mod.backward(sel, gD, 1.0)
    h = 1e-6

    def loss(X):
        DX, _ = oracle_mod.forward(X)
        return (gD * DX).sum() + DX[-1, -1]

    checked = 0
    for _ in range(40):
        i, j = rng.integers(0, 24, size=2)
        E = np.zeros_like(C)
        E[i, j] = h
        _, sp = oracle_mod.forward(C + E)
        _, sm = oracle_mod.forward(C - E)
        if not (np.array_equal(sp, sel) and np.array_equal(sm, sel)):
            continue  # a decision flips within +-h: the function is not differentiable there
        fd = (loss(C + E) - loss(C - E)) / (2 * h)
        assert abs(fd - gC[i, j]) <= 1e-6 * (1 + abs(gC[i, j]))
        checked += 1
    assert checked >= 30


def test_f32_adjoint_equals_f64_on_dyadic_data(oracle_mod):
    rng = np.random.default_rng(14)
    C = rng.integers(0, 64, size=(50, 60)).astype(np.float32)
    gD = rng.integers(-4, 5, size=(50, 60)).astype(np.float32)
    _, s32 = oracle_mod.forward(C, "f32")
    _, s64 = oracle_mod.forward(C, "f64")
    assert np.array_equal(s32, s64)
    g32 = oracle_mod.backward(s32, gD, 1.0, "f32")
    g64 = oracle_mod.backward(s64, gD, 1.0, "f64")
    assert np.array_equal(g32.astype(np.float64), g64)


def test_empty_and_degenerate(oracle_mod):
    D, sel = oracle_mod.forward(np.zeros((0, 5)))
    assert D.shape == (0, 5)
    D, sel = oracle_mod.forward(np.array([[2.5]]))
    assert D[0, 0] == 2.5 and sel[0, 0] == oracle_mod.SEL_NONE
    assert oracle_mod.backward(sel, None, 3.0)[0, 0] == 3.0
    # +inf marks a blocked cell; paths route around it
    C = np.array([[1.0, np.inf], [1.0, 1.0]])
    D, _ = oracle_mod.forward(C)
    assert D[1, 1] == 2.0 and np.isinf(D[0, 1])
