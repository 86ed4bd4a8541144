"""Tridiagonal linear systems -- test infrastructure only (oracle for the partition solver).

The paper's method solves a system A x = d whose coefficient matrix A is tridiagonal, of
size N, by the parallel partition method (Introduction): the rows are split into
sub-systems of m unknowns, each sub-system yields two interface equations, the interface
system (again tridiagonal, and diagonally dominant when A is) is solved, and the
sub-systems are then back-solved independently.  The recursive variant (section
"Recursive parallel partition method") solves the interface system by the same method
again, R times, with sub-system sizes m_1 .. m_R, before the last one is solved directly.

Two references live here:

- ``solve``: the plain definition x = A^-1 d, computed in float64 by Gaussian elimination
  without pivoting restricted to the three diagonals (the Thomas algorithm), which is
  stable for the diagonally dominant systems the paper treats.  The method reaches this
  solution up to rounding, so it is the reference for the solver's output.
- ``interface_system`` / ``back_solve`` / ``partition_solve``: the three stages written out
  in the order the Introduction gives them, so that the solver's intermediate results (the
  interface system of every level) can be checked too.  The paper names the stages but not
  their formulas (they come from the method's original source, which it cites); the
  formulas here are derived by block elimination, as stated in each function.  They are
  written over plain Python numbers, so that the tests can also run them in exact rational
  arithmetic (``fractions.Fraction``), where the method must give the exact solution.

Storage (the paper does not state one): three length-N arrays a (sub-diagonal, a[0] not
used), b (main diagonal), c (super-diagonal, c[N-1] not used), and the right-hand side d:
row i reads a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i].

Pure-Python loops: meant for the sizes the tests use (N up to about 1e6).
"""
from __future__ import annotations

import numpy as np


def solve(a, b, c, d) -> np.ndarray:
    """x with A x = d for the tridiagonal A given by its diagonals (float64)."""
    a, b, c, d = (np.asarray(v, dtype=np.float64) for v in (a, b, c, d))
    N = len(b)
    if not (len(a) == len(c) == len(d) == N) or N == 0:
        raise ValueError("a, b, c, d must have the same non-zero length")
    cp = np.zeros(N)  # super-diagonal of the eliminated (unit upper bidiagonal) system
    dp = np.zeros(N)  # its right-hand side
    # forward elimination: row i minus a[i] times the already normalised row i-1
    for i in range(N):
        piv = b[i] - (a[i] * cp[i - 1] if i > 0 else 0.0)
        if piv == 0.0:
            raise ZeroDivisionError(f"zero pivot in row {i}")
        cp[i] = c[i] / piv if i < N - 1 else 0.0
        dp[i] = (d[i] - (a[i] * dp[i - 1] if i > 0 else 0.0)) / piv
    # back substitution
    x = np.zeros(N)
    x[N - 1] = dp[N - 1]
    for i in range(N - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def dense(a, b, c) -> np.ndarray:
    """The N x N matrix the three diagonals describe."""
    N = len(b)
    A = np.zeros((N, N))
    for i in range(N):
        A[i, i] = b[i]
        if i > 0:
            A[i, i - 1] = a[i]
        if i < N - 1:
            A[i, i + 1] = c[i]
    return A


# ------------------------------------------------------------------------------------------
# The partition method, stage by stage.

def partition_sizes(N: int, m: int) -> list[tuple[int, int]]:
    """(first row, rows) of every sub-system of an N-row system cut into sub-systems of m rows.

    The paper cuts the N unknowns into sub-systems of m unknowns each and does not say what
    happens to a remainder.  Reading used here: ceil(N/m) sub-systems, all of m rows except
    the last, which holds the N - (ceil(N/m) - 1) m rows left over; a last sub-system of a
    single row joins the one before it (a sub-system needs two rows to own two interface
    unknowns).  Requires N >= 2 and m >= 2.
    """
    if N < 2 or m < 2:
        raise ValueError("the partition needs N >= 2 and m >= 2")
    P = -(-N // m)
    if P > 1 and N - (P - 1) * m == 1:
        P -= 1
    return [(k * m, m if k < P - 1 else N - (P - 1) * m) for k in range(P)]


def _eliminate_down(a, b, c, d, s, e):
    """Gaussian elimination of rows s+1 .. e of one sub-system, top to bottom, with x_s
    kept as an unknown of its own (a "spike").  Row s+1 is a[s+1] x_s + b x + c x = d; each
    next row i loses its x_{i-1} term by subtracting w = a[i]/p times the row above, which
    carries x_s along.  Returns the per-row coefficients (f_i on x_s, p_i on x_i, rhs q_i)
    for i = s+1 .. e: the eliminated row i reads f_i x_s + p_i x_i + c[i] x_{i+1} = q_i."""
    f, p, q = [a[s + 1]], [b[s + 1]], [d[s + 1]]
    for i in range(s + 2, e + 1):
        w = a[i] / p[-1]
        f.append(-w * f[-1])
        p.append(b[i] - w * c[i - 1])
        q.append(d[i] - w * q[-1])
    return f, p, q


def _eliminate_up(a, b, c, d, s, e):
    """The mirror image: elimination of rows e-1 .. s, bottom to top, with x_e kept as a
    spike.  Row e-1 is a x + b x + c[e-1] x_e = d; each next row i (going up) loses its
    x_{i+1} term by subtracting w = c[i]/r times the row below.  Returns the coefficients of
    the last row reached, row s: a[s] x_{s-1} + r x_s + g x_e = t."""
    g, r, t = c[e - 1], b[e - 1], d[e - 1]
    for i in range(e - 2, s - 1, -1):
        w = c[i] / r
        g = -w * g
        r = b[i] - w * a[i + 1]
        t = d[i] - w * t
    return g, r, t


def interface_system(a, b, c, d, m):
    """Stage 1: the interface system of the partition into sub-systems of m rows.

    For sub-system k with rows s .. e, its first and last unknowns x_s, x_e are its two
    interface unknowns; the interface system orders them z[2k] = x_s, z[2k+1] = x_e.  The
    two interface equations of the sub-system follow from eliminating its interior rows:
      - eliminating downward through rows s+1 .. e leaves an equation in x_s, x_e, x_{e+1}
        (the eliminated row e): row 2k+1 of the interface system;
      - eliminating upward through rows e-1 .. s leaves one in x_{s-1}, x_s, x_e (the
        eliminated row s): row 2k.
    x_{s-1} and x_{e+1} are the last and first unknowns of the neighbouring sub-systems, so
    the interface system is tridiagonal.  The terms outside the matrix (a[0], c[N-1]) are
    dropped.  Returns the interface system's diagonals and right-hand side (A, B, C, D), each
    of length 2P.
    """
    N = len(b)
    parts = partition_sizes(N, m)
    zero = b[0] - b[0]
    A, B, C, D = [], [], [], []
    for k, (s, L) in enumerate(parts):
        e = s + L - 1
        g, r, t = _eliminate_up(a, b, c, d, s, e)
        A.append(a[s] if k > 0 else zero)
        B.append(r)
        C.append(g)
        D.append(t)
        f, p, q = _eliminate_down(a, b, c, d, s, e)
        A.append(f[-1])
        B.append(p[-1])
        C.append(c[e] if k < len(parts) - 1 else zero)
        D.append(q[-1])
    return A, B, C, D


def back_solve(a, b, c, d, m, z):
    """Stage 3: with the interface unknowns z known (z[2k] = x_s, z[2k+1] = x_e), every
    sub-system's interior rows s+1 .. e-1 are an independent system.  Its downward
    elimination is the one of Stage 1 (recomputed); back substitution from x_e then gives
    x_i = (q_i - f_i x_s - c[i] x_{i+1}) / p_i for i = e-1 down to s+1."""
    N = len(b)
    x = [None] * N
    for k, (s, L) in enumerate(partition_sizes(N, m)):
        e = s + L - 1
        xs, xe = z[2 * k], z[2 * k + 1]
        x[s], x[e] = xs, xe
        f, p, q = _eliminate_down(a, b, c, d, s, e)
        for i in range(e - 1, s, -1):
            j = i - (s + 1)  # index of row i in the elimination's lists
            x[i] = (q[j] - f[j] * xs - c[i] * x[i + 1]) / p[j]
    return x


def thomas(a, b, c, d):
    """The Thomas algorithm over plain numbers (same steps as ``solve``), for Stage 2."""
    N = len(b)
    cp, dp = [None] * N, [None] * N
    for i in range(N):
        piv = b[i] - a[i] * cp[i - 1] if i > 0 else b[i]
        cp[i] = c[i] / piv if i < N - 1 else piv - piv
        dp[i] = (d[i] - a[i] * dp[i - 1]) / piv if i > 0 else d[i] / piv
    x = [None] * N
    x[N - 1] = dp[N - 1]
    for i in range(N - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def partition_levels(a, b, c, d, ms):
    """The interface systems of every level of the recursive method: level 0 is (a, b, c, d),
    level l+1 the interface system of level l cut into sub-systems of ms[l] rows."""
    levels = [(a, b, c, d)]
    for m in ms:
        levels.append(interface_system(*levels[-1], m))
    return levels


def partition_solve(a, b, c, d, ms):
    """The recursive partition method with sub-system sizes ms = [m, m_1, .., m_R] (R = the
    number of recursive steps; ms = [m] is the non-recursive method, ms = [] the direct
    solve).  Stage 1 on every level from the top, Stage 2 (Thomas) on the deepest interface
    system, Stage 3 on every level from the bottom.  A system of one row is solved directly
    at whatever level it appears."""
    as_float = isinstance(b, np.ndarray) or (len(b) and isinstance(b[0], float))
    a, b, c, d = (list(v) for v in (a, b, c, d))
    if len(b) == 0:
        raise ValueError("empty system")
    if len(b) == 1:
        ms = []
    levels = partition_levels(a, b, c, d, ms)
    z = thomas(*levels[-1])
    for lvl in range(len(ms) - 1, -1, -1):
        z = back_solve(*levels[lvl], ms[lvl], z)
    return np.asarray(z, dtype=np.float64) if as_float else z


# ------------------------------------------------------------------------------------------
# The same stages in plain C (oracle/tridiag.c), for sizes the loops above would take minutes
# on.  The tests hold them to the functions above bit for bit.

_PREC = {"f64": np.float64, "f32": np.float32}


def _c_arrays(vs, precision):
    t = _PREC[precision]
    return [np.ascontiguousarray(np.asarray(v), dtype=t) for v in vs]


def c_thomas(a, b, c, d, precision: str = "f64") -> np.ndarray:
    """``thomas`` in C, in float64 or float32 arithmetic."""
    from oracle import _load
    a, b, c, d = _c_arrays((a, b, c, d), precision)
    x = np.empty_like(b)
    if getattr(_load(), "tro_thomas_" + precision)(len(b), *(v.ctypes.data for v in (a, b, c, d, x))) != 0:
        raise MemoryError("oracle allocation failed")
    return x


def c_interface_system(a, b, c, d, m: int, precision: str = "f64"):
    """``interface_system`` in C: the arrays (A, B, C, D)."""
    from oracle import _load
    a, b, c, d = _c_arrays((a, b, c, d), precision)
    P = _load().tro_subsystems(len(b), m)
    if P < 0:
        raise ValueError("the partition needs N >= 2 and m >= 2")
    out = [np.empty(2 * P, dtype=b.dtype) for _ in range(4)]
    getattr(_load(), "tro_interface_" + precision)(len(b), m, *(v.ctypes.data for v in (a, b, c, d, *out)))
    return tuple(out)


def c_back_solve(a, b, c, d, m: int, z, precision: str = "f64") -> np.ndarray:
    """``back_solve`` in C."""
    from oracle import _load
    a, b, c, d, z = _c_arrays((a, b, c, d, z), precision)
    x = np.empty_like(b)
    if getattr(_load(), "tro_back_solve_" + precision)(len(b), m, *(v.ctypes.data for v in (a, b, c, d, z, x))):
        raise MemoryError("oracle allocation failed")
    return x


def c_partition_solve(a, b, c, d, ms, precision: str = "f64") -> np.ndarray:
    """``partition_solve`` in C; ms = [m, m_1, .., m_R] ([] = the direct solve)."""
    import ctypes
    from oracle import _load
    a, b, c, d = _c_arrays((a, b, c, d), precision)
    x = np.empty_like(b)
    R = len(ms) - 1
    arr = (ctypes.c_int32 * max(1, len(ms)))(*ms)
    rc = getattr(_load(), "tro_partition_" + precision)(len(b), R, arr, *(v.ctypes.data for v in (a, b, c, d, x)))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return x
