"""Pins for the oracle's substitutions (Eq. (3)), residual and backward error."""
import numpy as np
import pytest

import spdgen
from oracle import exact

U64 = 2.0 ** -53


def test_tridiagonal_inverse_closed_form(orc):
    # (T^{-1})_ij = min(i,j) (n+1-max(i,j)) / (n+1), 1-based
    n = 120
    L, info = orc.potrf(spdgen.tridiag(n))
    assert info == 0
    E = np.eye(n)  # columns e_k
    X = orc.potrs(L, E)  # (n, n): row k = T^{-1} e_k
    i = np.arange(1, n + 1)
    Tinv = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
    cond = 4.0 / (np.pi / (n + 1)) ** 2
    np.testing.assert_allclose(X, Tinv, atol=8 * cond * U64 * np.max(Tinv), rtol=0)


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_hilbert_inverse_integers(orc, n):
    H = spdgen.hilbert(n)
    L, info = orc.potrf(H)
    assert info == 0
    X = orc.potrs(L, np.eye(n))
    Hinv = np.array(exact.hilbert_inverse(n), dtype=np.float64)
    cond = np.linalg.cond(H)
    err = np.max(np.abs(X - Hinv)) / np.max(np.abs(Hinv))
    assert err <= 16 * n * cond * U64, err


@pytest.mark.parametrize("seed", [21, 22])
def test_exact_rational_solve(orc, seed):
    n = 8
    A = spdgen.logspaced(n, 1e5, seed)
    b = np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
    xe = np.array([float(v) for v in exact.solve(A, b)])
    x, info = orc.solve(A, b)
    assert info == 0
    err = np.max(np.abs(x[0] - xe)) / np.max(np.abs(xe))
    assert err <= 10 * 1e5 * U64 * n, err


@pytest.mark.parametrize("n,cond,m", [(200, 1e2, 1), (256, 1e4, 3), (180, 1e6, 2)])
def test_manufactured_solution(orc, n, cond, m):
    s = spdgen.system(n, cond, m, config=0, index=n)
    X, info = orc.solve(s.A, s.Bt)
    assert info == 0
    fwd = np.max(np.abs(X - s.Xt), axis=1) / np.max(np.abs(s.Xt), axis=1)
    assert np.all(fwd <= 10 * cond * U64), fwd
    eta = orc.backward_error(s.A, X, s.Bt)
    assert np.all(eta <= 4 * n * U64), eta


def test_forward_backward_substitution_separately(orc):
    # L = all-ones lower triangle (the min(i,j) factor): L^{-1} is the bidiagonal
    # [1, -1] difference operator, so L^{-1} b = first differences of b, exactly.
    n = 64
    L = np.tril(np.ones((n, n)))
    b = np.arange(1.0, n + 1.0) ** 2
    y = orc.fsub(L, b)[0]
    assert np.array_equal(y, np.diff(np.concatenate([[0.0], b])))
    # L^{-T} y = reversed first differences (backward)
    x = orc.bsub(L, y)[0]
    want = y - np.concatenate([y[1:], [0.0]])
    assert np.array_equal(x, want)


def test_residual_exact_on_integers(orc):
    # integer data small enough that every product and partial sum is exact
    rng = np.random.Generator(np.random.PCG64(5))
    n, m = 70, 3
    M = rng.integers(-9, 10, size=(n, n)).astype(np.float64)
    A = np.asfortranarray(M + M.T)
    X = rng.integers(-9, 10, size=(m, n)).astype(np.float64)
    B = rng.integers(-99, 100, size=(m, n)).astype(np.float64)
    R = orc.residual(A, X, B)
    Ai = A.astype(np.int64)
    want = B.astype(np.int64) - (Ai @ X.T.astype(np.int64)).T
    assert np.array_equal(R, want.astype(np.float64))
    # only the lower triangle is used
    Ap = A.copy(order="F")
    Ap[np.triu_indices(n, 1)] = 1e300
    assert np.array_equal(orc.residual(Ap, X, B), R)
    rows = np.array([0, 17, n - 1])
    assert np.array_equal(orc.residual_rows(A, X, B, rows), R[:, rows])


def test_backward_error_closed_form(orc):
    # A = min(i,j), x integer, b = A x exactly -> eta = 0; perturb x_k by 2^-10
    # -> r = -2^-10 A e_k exactly, ||r||_inf = 2^-10 * n (last row of column k... max_i min(i,k) = k)
    n = 32
    A = spdgen.minij(n)
    x = np.arange(1.0, n + 1.0)
    b = A @ x
    assert orc.backward_error(A, x, b)[0] == 0.0
    k = 10  # 1-based column
    xp = x.copy()
    xp[k - 1] += 2.0 ** -10
    eta = orc.backward_error(A, xp, b)[0]
    anorm = float(sum(min(n, j) for j in range(1, n + 1)))  # row n sums to n(n+1)/2
    assert orc.norminf_sym(A) == anorm
    want = (2.0 ** -10 * k) / (anorm * np.max(np.abs(xp)) + np.max(np.abs(b)))
    assert eta == pytest.approx(want, rel=4 * U64)


def test_backward_error_nan(orc):
    A = spdgen.minij(8)
    x = np.ones(8)
    x[3] = np.nan
    assert np.isnan(orc.backward_error(A, x, A @ np.ones(8))[0])


def test_golden_exact_small(orc):
    import json
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "exact_small.json")
    with open(path) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        n = c["n"]
        A = np.asfortranarray(np.array(c["A"], dtype=np.float64))
        b = np.array(c["b"], dtype=np.float64)
        L, info = orc.potrf(A)
        assert info == 0
        for i in range(n):
            for j in range(i + 1):
                want = c["L_sign"][i][j] * float(Fraction(c["L_squared"][i][j])) ** 0.5
                assert abs(L[i, j] - want) <= 32 * U64 * max(1.0, abs(want)), (n, i, j)
        x, info = orc.solve(A, b)
        xe = np.array([float(Fraction(v)) for v in c["x"]])
        cond = np.linalg.cond(A)
        assert np.max(np.abs(x[0] - xe)) <= 10 * cond * U64 * np.max(np.abs(xe)) * n


def test_residual_given_rows_matches_full_residual(orc):
    # the rows-only residual is the full residual restricted to those rows
    s = spdgen.system(90, 1e3, 2, config=0, index=21)
    X = s.Xt + 1e-6
    rows = np.array([0, 7, 45, 89])
    R = orc.residual(s.A, X, s.Bt)
    Rg = orc.residual_given_rows(s.A[rows, :], X, s.Bt, rows)
    assert np.array_equal(Rg, R[:, rows])


def test_logspaced_kron_generator_spectrum():
    # the large-order recipe (no order-n QR): exactly symmetric, dense, and
    # its eigenvalues are the log-spaced lambda_i = cond^((i-1)/(n-1))
    import torch
    n, cond = 12 * 16, 1e5
    A = spdgen.logspaced_kron(n, cond, 5, device="cpu", chunk=50).numpy()
    assert np.array_equal(A, A.T)
    assert np.count_nonzero(A) == n * n
    lam = np.linalg.eigvalsh(A)
    want = cond ** (np.arange(n) / (n - 1))
    assert np.abs(lam - want).max() <= 1e-13 * cond
    # seeded: the same call gives the same bytes
    B = spdgen.logspaced_kron(n, cond, 5, device="cpu", chunk=64).numpy()
    assert np.array_equal(A, B)
