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
