"""Tridiagonal linear systems -- test infrastructure only (oracle for the partition solver).

The paper's method solves a system A x = d whose coefficient matrix A is tridiagonal, of
size N, by the parallel partition method (Introduction): the rows are split into
sub-systems of m unknowns, each sub-system yields two interface equations, the interface
system (again tridiagonal, and diagonally dominant when A is) is solved, and the
sub-systems are then back-solved independently.  The method reaches the exact solution up
to rounding, so the oracle is the plain definition x = A^-1 d, computed in float64 by
Gaussian elimination without pivoting restricted to the three diagonals (the Thomas
algorithm), which is stable for the diagonally dominant systems the paper treats.

Storage (the paper does not state one): three length-N arrays a (sub-diagonal, a[0] not
used), b (main diagonal), c (super-diagonal, c[N-1] not used), and the right-hand side d:
row i reads a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i].

Pure-Python loops: meant for the sizes the tests use (N up to about 1e5).
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
