"""Exact rational references for tiny systems -- TEST INFRASTRUCTURE ONLY.

Every binary64 input is converted to the exact rational it denotes
(``fractions.Fraction(float)`` is exact), so these results carry no rounding
at all and pin the binary64 oracle from outside.

* ``ldlt(A)``: A = L D L^T with unit lower L, found by Gaussian elimination in
  exact arithmetic.  The Cholesky factor of Section 3.1 is L diag(sqrt(D)),
  so ``L_chol[i][j]^2 = L[i][j]^2 * D[j]`` exactly, and the first j with
  D[j] <= 0 is the column where Cholesky breaks down.
* ``solve(A, b)``: exact Gaussian elimination (no pivoting is needed for SPD).
* ``hilbert_inverse(n)``: the classical closed form of the Hilbert inverse.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb


def _frac_matrix(A):
    n = len(A)
    return [[Fraction(float(A[i][j])) for j in range(n)] for i in range(n)]


def ldlt(A):
    """Exact A = L D L^T.  Returns (L, D, first_nonpositive_1based_or_0)."""
    M = _frac_matrix(A)
    n = len(M)
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    D = [Fraction(0)] * n
    fail = 0
    for j in range(n):
        D[j] = M[j][j] - sum(L[j][k] ** 2 * D[k] for k in range(j))
        if D[j] <= 0:
            fail = j + 1
            break
        for i in range(j + 1, n):
            L[i][j] = (M[i][j] - sum(L[i][k] * L[j][k] * D[k] for k in range(j))) / D[j]
    return L, D, fail


def solve(A, b):
    """Exact solution of A x = b by Gaussian elimination (A nonsingular, no pivoting)."""
    M = _frac_matrix(A)
    n = len(M)
    v = [Fraction(float(x)) for x in b]
    for k in range(n):
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            for j in range(k, n):
                M[i][j] -= f * M[k][j]
            v[i] -= f * v[k]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (v[i] - sum(M[i][j] * x[j] for j in range(i + 1, n))) / M[i][i]
    return x


def hilbert_inverse(n):
    """(H^{-1})_ij = (-1)^{i+j} (i+j-1) C(n+i-1, n-j) C(n+j-1, n-i) C(i+j-2, i-1)^2, 1-based."""
    out = [[0] * n for _ in range(n)]
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            out[i - 1][j - 1] = ((-1) ** (i + j) * (i + j - 1) * comb(n + i - 1, n - j)
                                 * comb(n + j - 1, n - i) * comb(i + j - 2, i - 1) ** 2)
    return out
