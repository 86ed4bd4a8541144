"""Pins of the tridiagonal-system oracle (the reference for the partition solver): no GPU."""
import numpy as np
import pytest

from oracle import tridiag
from paper_2510_27351_amd import inputs


def _system(N, seed):
    return tuple(v.numpy() for v in inputs.tridiagonal_dd(N, seed))


def _band_product(a, b, c, x):
    """A x from the diagonals, row by row (row i: a[i] x[i-1] + b[i] x[i] + c[i] x[i+1])."""
    N = len(x)
    y = b * x
    y[1:] += a[1:] * x[:-1]
    y[:-1] += c[:-1] * x[1:]
    return y


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 257])
def test_matches_dense_library_solve(N):
    a, b, c, d = _system(N, seed=N)
    x = tridiag.solve(a, b, c, d)
    ref = np.linalg.solve(tridiag.dense(a, b, c), d)
    assert np.max(np.abs(x - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_dense_matrix_layout():
    A = tridiag.dense([0.0, 1.0, 2.0], [4.0, 5.0, 6.0], [7.0, 8.0, 0.0])
    assert np.array_equal(A, [[4, 7, 0], [1, 5, 8], [0, 2, 6]])


@pytest.mark.parametrize("N", [10, 1000, 20000])
def test_manufactured_solution(N):
    """Pick x, form d = A x from the diagonals, solve: x comes back within a bound set by the
    conditioning.  Dominance by a margin of 1 gives ||A^-1||_inf <= 1, the rows of |A| sum to
    at most 6, so a backward-stable solve plus the rounding of d = A x leave an error of a
    few units in the last place times 6; 256 ulps is the bound used."""
    a, b, c, _ = _system(N, seed=100 + N)
    x = np.random.default_rng(N).uniform(-1, 1, N)
    got = tridiag.solve(a, b, c, _band_product(a, b, c, x))
    assert np.max(np.abs(got - x)) <= 64 * np.finfo(np.float64).eps * 4


def test_diagonal_system_is_exact():
    a, b, c, d = _system(500, seed=7)
    z = np.zeros_like(a)
    assert np.array_equal(tridiag.solve(z, b, z, d), d / b)


def test_two_by_two_closed_form():
    """Cramer's rule for [[b0, c0], [a1, b1]] x = d."""
    a, b, c, d = [0.0, 1.5], [4.0, -3.0], [2.0, 0.0], [1.0, 2.0]
    det = b[0] * b[1] - c[0] * a[1]
    want = [(d[0] * b[1] - c[0] * d[1]) / det, (b[0] * d[1] - a[1] * d[0]) / det]
    assert np.allclose(tridiag.solve(a, b, c, d), want, rtol=1e-15, atol=0)


def test_constant_coefficients_closed_form():
    """-x[i-1] + 2 x[i] - x[i+1] = h^2 f with x = 0 outside [1, N]: for f = 1 the exact solution
    of the discrete problem is x[i] = h^2 i (N + 1 - i) / 2 (i = 1..N)."""
    N = 99
    h = 1.0 / (N + 1)
    a, b, c = -np.ones(N), 2 * np.ones(N), -np.ones(N)
    a[0] = c[-1] = 0.0
    i = np.arange(1, N + 1)
    want = h * h * i * (N + 1 - i) / 2
    got = tridiag.solve(a, b, c, h * h * np.ones(N))
    assert np.max(np.abs(got - want)) <= 1e-12


def test_generator_is_diagonally_dominant():
    a, b, c, _ = _system(4096, seed=3)
    assert a[0] == 0.0 and c[-1] == 0.0
    assert np.all(np.abs(b) >= np.abs(a) + np.abs(c) + 1.0)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        tridiag.solve([0.0], [1.0, 2.0], [0.0], [1.0])
    with pytest.raises(ZeroDivisionError):
        tridiag.solve([0.0, 1.0], [0.0, 1.0], [1.0, 0.0], [1.0, 1.0])


# Plausible mistakes planted in a private copy of the oracle's source; the dense-solve pin must
# reject each one.  The shipped oracle is never modified.
MUTATIONS = {
    "back_substitution_sign": ("x[i] = dp[i] - cp[i] * x[i + 1]", "x[i] = dp[i] + cp[i] * x[i + 1]"),
    "pivot_wrong_index": ("piv = b[i] - (a[i] * cp[i - 1] if i > 0 else 0.0)",
                          "piv = b[i] - (a[i] * cp[i] if i > 0 else 0.0)"),
    "pivot_dropped_term": ("piv = b[i] - (a[i] * cp[i - 1] if i > 0 else 0.0)", "piv = b[i]"),
    "rhs_transposed_diagonal": ("dp[i] = (d[i] - (a[i] * dp[i - 1] if i > 0 else 0.0)) / piv",
                                "dp[i] = (d[i] - (c[i] * dp[i - 1] if i > 0 else 0.0)) / piv"),
    "super_diagonal_shift": ("cp[i] = c[i] / piv if i < N - 1 else 0.0",
                             "cp[i] = c[i - 1] / piv if i < N - 1 else 0.0"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistakes(name):
    import inspect
    old, new = MUTATIONS[name]
    src = inspect.getsource(tridiag.solve)
    assert src.count(old) == 1, name
    scope = {"np": np}
    exec(src.replace(old, new), scope)
    mutated = scope["solve"]
    a, b, c, d = _system(50, seed=9)
    x = mutated(a, b, c, d)
    ref = np.linalg.solve(tridiag.dense(a, b, c), d)
    assert np.max(np.abs(x - ref)) > 1e-6, name


# ------------------------------------------------------------------------------------------
# The partition method, stage by stage (tridiag.interface_system / back_solve /
# partition_solve): pinned to exact rational arithmetic, to the dense solve, and to the
# properties the paper states for the interface system.

from fractions import Fraction


def _rational_system(N, seed):
    """A diagonally dominant system with small-integer-ratio rational entries."""
    rng = np.random.default_rng(seed)
    a = [Fraction(int(v), 4) for v in rng.integers(-4, 5, N)]
    c = [Fraction(int(v), 4) for v in rng.integers(-4, 5, N)]
    a[0] = Fraction(0)
    c[N - 1] = Fraction(0)
    b = [(abs(a[i]) + abs(c[i]) + 1 + Fraction(int(rng.integers(0, 8)), 8)) * (1 if rng.random() < 0.5 else -1)
         for i in range(N)]
    d = [Fraction(int(v), 3) for v in rng.integers(-9, 10, N)]
    return a, b, c, d


def _exact_residual_is_zero(a, b, c, d, x):
    N = len(b)
    for i in range(N):
        s = b[i] * x[i]
        if i > 0:
            s += a[i] * x[i - 1]
        if i < N - 1:
            s += c[i] * x[i + 1]
        if s != d[i]:
            return False
    return True


@pytest.mark.parametrize("N,ms", [(2, [2]), (3, [2]), (13, [4]), (13, [3]), (17, [5]), (40, [4, 3]),
                                  (41, [6, 4, 2]), (64, [8, 10, 4]), (9, [9]), (9, [20])])
def test_partition_exact_in_rationals(N, ms):
    """In exact arithmetic the method returns the exact solution: A x = d holds exactly."""
    a, b, c, d = _rational_system(N, seed=N * 7 + len(ms))
    x = tridiag.partition_solve(a, b, c, d, ms)
    assert all(isinstance(v, Fraction) for v in x)
    assert _exact_residual_is_zero(a, b, c, d, x)


def test_partition_interface_exact_in_rationals():
    """Every interface equation holds exactly for the exact solution, and the interface
    system's own solution is the full solution at the interface unknowns (section on the
    three stages: solving the interface system finds some of the unknowns)."""
    a, b, c, d = _rational_system(23, seed=5)
    x = tridiag.thomas(a, b, c, d)
    assert _exact_residual_is_zero(a, b, c, d, x)
    A, B, C, D = tridiag.interface_system(a, b, c, d, 5)
    parts = tridiag.partition_sizes(23, 5)
    zx = []
    for s, L in parts:
        zx += [x[s], x[s + L - 1]]
    assert _exact_residual_is_zero(A, B, C, D, zx)
    assert tridiag.thomas(A, B, C, D) == zx


@pytest.mark.parametrize("N,m,want", [
    (10, 5, [(0, 5), (5, 5)]), (11, 5, [(0, 5), (5, 6)]), (12, 5, [(0, 5), (5, 5), (10, 2)]),
    (2, 2, [(0, 2)]), (3, 2, [(0, 3)]), (5, 8, [(0, 5)]), (7, 3, [(0, 3), (3, 4)])])
def test_partition_sizes(N, m, want):
    assert tridiag.partition_sizes(N, m) == want


def test_partition_sizes_rejects():
    with pytest.raises(ValueError):
        tridiag.partition_sizes(1, 4)
    with pytest.raises(ValueError):
        tridiag.partition_sizes(10, 1)


@pytest.mark.parametrize("N,ms", [(1, [4]), (2, [2]), (100, [4]), (1000, [32]), (1001, [32]), (999, [7, 10]),
                                  (5000, [64, 10, 16]), (4097, [16, 10, 8, 4])])
def test_partition_matches_dense_solve(N, ms):
    a, b, c, d = _system(N, seed=200 + N)
    x = tridiag.partition_solve(a, b, c, d, ms)
    ref = np.linalg.solve(tridiag.dense(a, b, c), d)
    assert np.max(np.abs(x - ref)) <= 1e-13


def test_interface_system_is_diagonally_dominant():
    """The paper: the interface system is tridiagonal, and diagonally dominant when the
    initial one is.  Checked on random dominant systems, every level of a recursion."""
    a, b, c, d = _system(6000, seed=11)
    for lvl, (A, B, C, D) in enumerate(tridiag.partition_levels(a, b, c, d, [32, 10, 8])):
        A, B, C = (np.asarray(v, dtype=np.float64) for v in (A, B, C))
        assert A[0] == 0.0 and C[-1] == 0.0, lvl
        assert np.all(np.abs(B) > np.abs(A) + np.abs(C)), lvl


def test_interface_equations_hold_for_the_solution():
    """Float64: every interface equation's residual at the true solution is at rounding level."""
    N, m = 3000, 24
    a, b, c, d = _system(N, seed=12)
    x = np.linalg.solve(tridiag.dense(a, b, c), d)
    A, B, C, D = (np.asarray(v, dtype=np.float64) for v in tridiag.interface_system(a, b, c, d, m))
    z = np.array([x[i] for s, L in tridiag.partition_sizes(N, m) for i in (s, s + L - 1)])
    r = B * z - D
    r[1:] += A[1:] * z[:-1]
    r[:-1] += C[:-1] * z[1:]
    assert np.max(np.abs(r)) <= 1e-13 * np.max(np.abs(B))


def test_partition_with_m_two_keeps_the_rows():
    """m = 2: no interior rows, so the interface system is the original system itself."""
    a, b, c, d = _system(50, seed=13)
    A, B, C, D = tridiag.interface_system(a, b, c, d, 2)
    assert np.array_equal(np.asarray(A), a) and np.array_equal(np.asarray(B), b)
    assert np.array_equal(np.asarray(C), c) and np.array_equal(np.asarray(D), d)


PARTITION_MUTATIONS = {
    "down_spike_sign": ("f.append(-w * f[-1])", "f.append(w * f[-1])"),
    "down_wrong_upper": ("p.append(b[i] - w * c[i - 1])", "p.append(b[i] - w * c[i])"),
    "up_dropped_rhs_term": ("t = d[i] - w * t", "t = d[i]"),
    "up_wrong_lower": ("r = b[i] - w * a[i + 1]", "r = b[i] - w * a[i]"),
    "up_start_row": ("g, r, t = c[e - 1], b[e - 1], d[e - 1]", "g, r, t = c[e - 1], b[e - 1], d[e]"),
    "back_spike_sign": ("x[i] = (q[j] - f[j] * xs - c[i] * x[i + 1]) / p[j]",
                        "x[i] = (q[j] + f[j] * xs - c[i] * x[i + 1]) / p[j]"),
    "interface_lower_from_wrong_row": ("A.append(a[s] if k > 0 else zero)", "A.append(a[s + 1] if k > 0 else zero)"),
}


@pytest.mark.parametrize("name", sorted(PARTITION_MUTATIONS))
def test_partition_pins_catch_planted_mistakes(name):
    """Plausible mistakes planted in a private copy of the stage functions: the exact
    rational pin and the dense-solve pin must both reject each one."""
    import inspect
    import types
    old, new = PARTITION_MUTATIONS[name]
    src = inspect.getsource(tridiag)
    assert src.count(old) == 1, name
    mod = types.ModuleType("tridiag_mutated")
    exec(compile(src.replace(old, new), "tridiag_mutated", "exec"), mod.__dict__)
    a, b, c, d = _rational_system(17, seed=3)
    try:
        x = mod.partition_solve(a, b, c, d, [5])
        assert not _exact_residual_is_zero(a, b, c, d, x), name
    except ZeroDivisionError:
        pass
    a, b, c, d = _system(300, seed=4)
    x = mod.partition_solve(a, b, c, d, [12])
    ref = np.linalg.solve(tridiag.dense(a, b, c), d)
    assert np.max(np.abs(x - ref)) > 1e-8, name


# ------------------------------------------------------------------------------------------
# The C twin of the stages (oracle/tridiag.c), used for the large GPU parity cases: equal to
# the Python stages bit for bit, in float64 and in float32 (Python loops over np.float32
# scalars round every operation to float32, as the C float code does).

C_CASES = [(1, []), (2, [2]), (3, [2]), (10, [4]), (11, [5]), (101, [8, 10]), (1000, [16, 10, 4]),
           (4097, [64]), (20001, [32, 10, 8, 4]), (3000, [37, 3])]


def _f32(v):
    return [np.float32(x) for x in np.asarray(v, dtype=np.float32)]


@pytest.mark.parametrize("N,ms", C_CASES)
def test_c_partition_equals_python_f64(N, ms):
    a, b, c, d = _system(N, seed=N)
    assert np.array_equal(tridiag.c_partition_solve(a, b, c, d, ms), tridiag.partition_solve(a, b, c, d, ms))


@pytest.mark.parametrize("N,ms", C_CASES)
def test_c_partition_equals_python_f32(N, ms):
    a, b, c, d = _system(N, seed=N + 1)
    want = np.asarray(tridiag.partition_solve(_f32(a), _f32(b), _f32(c), _f32(d), ms), dtype=np.float32)
    assert np.array_equal(tridiag.c_partition_solve(a, b, c, d, ms, "f32"), want)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N,m", [(2, 2), (9, 4), (10, 4), (1001, 32), (515, 256)])
def test_c_stages_equal_python(N, m, precision):
    a, b, c, d = _system(N, seed=2 * N + m)
    conv = (lambda v: list(v)) if precision == "f64" else _f32
    t = np.float64 if precision == "f64" else np.float32
    want = tridiag.interface_system(conv(a), conv(b), conv(c), conv(d), m)
    got = tridiag.c_interface_system(a, b, c, d, m, precision)
    for g, w in zip(got, want):
        assert np.array_equal(g, np.asarray(w, dtype=t))
    z = tridiag.c_thomas(*got, precision)
    assert np.array_equal(z, np.asarray(tridiag.thomas(*(conv(v) for v in got)), dtype=t))
    x = tridiag.c_back_solve(a, b, c, d, m, z, precision)
    assert np.array_equal(x, np.asarray(tridiag.back_solve(conv(a), conv(b), conv(c), conv(d), m, conv(z)), dtype=t))


def test_c_thomas_equals_solve():
    a, b, c, d = _system(5000, seed=9)
    assert np.array_equal(tridiag.c_thomas(a, b, c, d), tridiag.solve(a, b, c, d))
