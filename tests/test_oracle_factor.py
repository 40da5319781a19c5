"""Pins for the oracle's Cholesky factorisation (Section 3.1: A = R^T R, here L = R^T).

Each test ties the oracle to something other than itself: a closed form, an
exact rational factorisation, a structural invariant, or the textbook bound.
"""
import numpy as np
import pytest

import spdgen
from oracle import exact

U64 = 2.0 ** -53


def test_tridiagonal_closed_form(orc):
    # [-1, 2, -1]: L_ii = sqrt((i+1)/i), L_{i+1,i} = -sqrt(i/(i+1))  (1-based i)
    n = 300
    L, info = orc.potrf(spdgen.tridiag(n))
    assert info == 0
    i = np.arange(1, n + 1, dtype=np.float64)
    diag = np.sqrt((i + 1) / i)
    sub = -np.sqrt(i[:-1] / (i[:-1] + 1))
    np.testing.assert_allclose(np.diag(L), diag, rtol=8 * U64 * 4, atol=0)
    np.testing.assert_allclose(np.diag(L, -1), sub, rtol=8 * U64 * 4, atol=0)
    # everything else in the lower triangle is exactly zero (no fill-in)
    assert np.count_nonzero(np.tril(L, -2)) == 0
    assert np.count_nonzero(np.triu(L, 1)) == 0


def test_minij_factor_is_all_ones(orc):
    # a_ij = min(i, j): L is exactly the all-ones lower triangle (every step exact)
    n = 257
    L, info = orc.potrf(spdgen.minij(n))
    assert info == 0
    assert np.array_equal(L, np.tril(np.ones((n, n))))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_exact_rational_ldlt_small(orc, seed):
    # n <= 8: exact A = L D L^T, so L_chol[i][j]^2 = L[i][j]^2 * D[j] exactly
    n = 7
    A = spdgen.logspaced(n, 1e3, seed)
    Lx, D, fail = exact.ldlt(A)
    assert fail == 0
    L, info = orc.potrf(A)
    assert info == 0
    scale = np.max(np.abs(L))
    for i in range(n):
        for j in range(i + 1):
            sq = Lx[i][j] ** 2 * D[j]          # exact square of the true entry
            want = float(np.sign(float(Lx[i][j]))) * float(sq) ** 0.5
            assert abs(L[i, j] - want) <= 1e3 * 64 * U64 * scale, (i, j, L[i, j], want)
            if i == j:
                assert L[i, i] > 0
    # strictly upper part is zero
    assert np.count_nonzero(np.triu(L, 1)) == 0


def test_hilbert_exact_ldlt(orc):
    n = 6
    A = spdgen.hilbert(n)
    Lx, D, fail = exact.ldlt(A)
    assert fail == 0
    L, info = orc.potrf(A)
    assert info == 0
    got = np.diag(L) ** 2
    want = np.array([float(d) for d in D])
    # cond(H6) ~ 1.5e7: pivots are still accurate to ~cond * u
    np.testing.assert_allclose(got, want, rtol=1.5e7 * 64 * U64)


@pytest.mark.parametrize("n,cond", [(64, 1e2), (200, 1e4), (333, 1e6)])
def test_backward_error_invariant(orc, n, cond):
    A = spdgen.logspaced(n, cond, 11 + n)
    L, info = orc.potrf(A)
    assert info == 0
    E = A - L @ L.T
    rel = np.linalg.norm(E) / np.linalg.norm(A)
    assert rel <= 4 * n * U64, rel
    # componentwise form of the classical bound |A - L L^T| <= gamma_{n+1} |L||L^T|
    bound = (n + 1) * U64 / (1 - (n + 1) * U64) * (np.abs(L) @ np.abs(L.T))
    assert np.all(np.abs(E) <= bound + 1e-300)
    # the positive-diagonal Cholesky factor is unique: a library factor agrees
    Lref = np.linalg.cholesky(A)
    assert np.max(np.abs(L - Lref)) <= 1e3 * cond ** 0.5 * U64 * np.max(np.abs(L))


def test_only_lower_triangle_is_read(orc):
    n = 50
    A = spdgen.logspaced(n, 1e3, 5)
    Ag = A.copy(order="F")
    Ag[np.triu_indices(n, 1)] = np.nan  # poison the strict upper triangle
    L1, i1 = orc.potrf(A)
    L2, i2 = orc.potrf(Ag)
    assert i1 == i2 == 0
    assert np.array_equal(L1, L2)


@pytest.mark.parametrize("n,j0", [(9, 1), (9, 4), (40, 17), (64, 64)])
def test_indefinite_reports_first_failing_column(orc, n, j0):
    A = spdgen.indefinite(n, j0)
    if n <= 9:
        _, _, fail = exact.ldlt(A)
        assert fail == j0
    _, info = orc.potrf(A)
    assert info == j0


def test_nan_input_fails(orc):
    A = spdgen.logspaced(20, 10.0, 3)
    A[5, 5] = np.nan
    _, info = orc.potrf(A)
    assert info == 6


def test_covariance_matrix_is_spd(orc):
    # Section 4 model covariance; for d in {1,2,4} the Toeplitz part's symbol is
    # bounded below by -2 ln 2, -pi^2/6, -(7/4) zeta(4) > -2 >= -min diag, so SPD.
    for d in (1, 2, 4):
        A = spdgen.covariance(400, d)
        _, info = orc.potrf(A)
        assert info == 0
        lam = np.linalg.eigvalsh(A)
        assert lam[0] > 2.0 - 2.0 * np.log(2.0) - 1e-9 if d == 1 else lam[0] > 0
