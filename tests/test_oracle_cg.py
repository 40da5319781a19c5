"""Pins of the oracle's Algorithm 2 (CG with iterative refinement,
Section 3.2; banded operator of Section 4) against what the mathematics
fixes, independently of the oracle's own code:

* after k products, CG's iterate is the minimiser of the A-norm error over
  the Krylov space K_k(A, b), computed here from an explicit basis;
* on a matrix with three distinct eigenvalues CG stops after three products;
* with the inner solve run to the end, one outer step gives x0 + A~^{-1} r0
  for A~ = fl32(A) kept on the band |i - j| <= k (a wrong band fails it);
* refinement reaches eta <= 1e-14 on the covariance matrices of Section 4,
  dense and banded (half-band 16), with the forward error inside the
  normwise bound 2 (eta + u) kappa_inf(A) that this backward error implies;
* a banded operator for which Eq. (4) fails diverges, and is reported;
* columns run in lockstep but do not influence one another.
"""
import numpy as np
import pytest

import spdgen

U64 = 2.0 ** -53


def _int_spd(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    G = rng.integers(-3, 4, size=(n, n)).astype(np.float64)
    return np.asfortranarray(G @ G.T + 4.0 * n * np.eye(n))


def _krylov_min(A, b, k):
    """argmin over x in K_k(A, b) of ||x - A^{-1} b||_A, from an orthonormal basis."""
    n = len(b)
    V = np.zeros((n, k))
    v = b / np.linalg.norm(b)
    for j in range(k):
        for _ in range(2):  # Gram-Schmidt, twice
            v = v - V[:, :j] @ (V[:, :j].T @ v)
        V[:, j] = v / np.linalg.norm(v)
        v = A @ V[:, j]
    H = V.T @ A @ V
    return V @ np.linalg.solve(H, V.T @ b)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_cg_iterate_is_krylov_minimiser(orc, k):
    n = 16
    A = _int_spd(n, 3)
    b = np.arange(1, n + 1, dtype=np.float64) * np.where(np.arange(n) % 2, 1.0, -1.0)
    X, rep = orc.cg_ir(A, b, max_outer=1, max_inner=k, inner_tol=0.0)
    assert rep.iters_low == k and rep.iters_high == 2
    xk = _krylov_min(A, b, k)
    assert np.abs(X[0] - xk).max() <= 1e-5 * np.abs(xk).max()


def test_cg_three_distinct_eigenvalues_three_products(orc):
    n = 30
    lam = np.array([1.0, 2.0, 4.0])[np.arange(n) % 3]
    A = np.asfortranarray(np.diag(lam))
    b = np.ones(n)
    X, rep = orc.cg_ir(A, b, max_outer=1, inner_tol=1e-6)
    assert rep.iters_low == 3
    assert np.abs(X[0] - b / lam).max() <= 1e-6


@pytest.mark.parametrize("k", [0, 2, 5])
def test_one_outer_step_is_banded_solve(orc, k):
    n = 60
    A = spdgen.covariance(n, 1)
    b = spdgen.rhs(n, 1, 11)[0]
    X, rep = orc.cg_ir(A, b, half_band=k, max_outer=1, max_inner=500, inner_tol=1e-12)
    At = A.astype(np.float32).astype(np.float64)
    i, j = np.indices((n, n))
    At[np.abs(i - j) > k] = 0.0
    x1 = np.linalg.solve(At, b)
    assert np.abs(X[0] - x1).max() <= 1e-5 * np.abs(x1).max()
    # the neighbouring band widths give visibly different steps
    for kk in (k + 1,) + ((k - 1,) if k > 0 else ()):
        Ak = A.copy()
        Ak[np.abs(i - j) > kk] = 0.0
        assert np.abs(np.linalg.solve(Ak, b) - x1).max() > 1e-3 * np.abs(x1).max()


@pytest.mark.parametrize("d", [1, 2, 4])
@pytest.mark.parametrize("band", [-1, 16])
def test_cg_ir_converges_on_covariance(orc, d, band):
    n, m = 300, 2
    A = spdgen.covariance(n, d)
    Xt = spdgen.rhs(n, m, 5 + d)
    Bt = spdgen.accurate_product(A, Xt)
    X, rep = orc.cg_ir(A, Bt, half_band=band)
    assert rep.status == 0 and rep.iters_high >= 2
    eta = orc.backward_error(A, X, Bt).max()
    assert eta <= 1e-14
    # normwise forward-error bound for a backward error eta (B itself rounded once)
    kinf = np.abs(A).sum(axis=1).max() * np.abs(np.linalg.inv(A)).sum(axis=1).max()
    fe = (np.abs(X - Xt).max(axis=1) / np.abs(Xt).max(axis=1)).max()
    assert fe <= 2 * (eta + U64) * kinf


def test_band_violating_eq4_diverges(orc):
    # A = (1-a) I + a 11^T: with the diagonal alone (half-band 0) the outer
    # iteration multiplies the error by I - A~^{-1} A, whose eigenvalue
    # -(n-1) a has modulus 2.9 > 1.
    n, a = 30, 0.1
    A = np.asfortranarray((1 - a) * np.eye(n) + a * np.ones((n, n)))
    b = spdgen.rhs(n, 1, 3)[0]
    _, rep = orc.cg_ir(A, b, half_band=0)
    assert rep.status == 3
    X, rep = orc.cg_ir(A, b)
    assert rep.status == 0 and orc.backward_error(A, X, b).max() <= 1e-14


def test_columns_are_independent(orc):
    n = 80
    A = spdgen.covariance(n, 2)
    Bt = spdgen.rhs(n, 3, 21)
    X, rep = orc.cg_ir(A, Bt, half_band=4)
    for c in range(3):
        Xc, _ = orc.cg_ir(A, Bt[c], half_band=4)
        assert np.array_equal(Xc[0], X[c])


def test_zero_rhs(orc):
    A = spdgen.covariance(20, 1)
    X, rep = orc.cg_ir(A, np.zeros(20))
    assert rep.status == 0 and rep.iters_low == 0 and rep.iters_high == 1 and rep.eta == 0.0
    assert not X.any()


@pytest.mark.parametrize("n,d,k", [(200, 1, 0), (200, 1, 1), (200, 1, 3), (200, 1, 8), (120, 1, 2),
                                   (200, 2, 1), (200, 2, 2), (200, 2, 8)])
def test_outer_contraction_follows_the_spectral_radius(orc, n, d, k):
    """With the inner solve run to the end, each outer step multiplies the
    error by I - A~^{-1} A.  Refinement therefore diverges when that matrix's
    spectral radius rho exceeds 1, and otherwise needs about
    1 + ln(1/tol) / ln(1/rho) residuals from x0 = 0 (eta_1 = 1).  Where
    Eq. (4)'s sufficient condition ||A^{-1} (A - A~)||_inf < 1 holds, it
    converges.  rho and the norm come from numpy, not from the oracle."""
    A = spdgen.covariance(n, d)
    i, j = np.indices((n, n))
    At = A.astype(np.float32).astype(np.float64)
    At[np.abs(i - j) > k] = 0.0
    rho = max(abs(np.linalg.eigvals(np.eye(n) - np.linalg.solve(At, A))))
    eq4 = np.abs(np.linalg.solve(A, A - At)).sum(axis=1).max()
    b = spdgen.rhs(n, 1, 5)[0]
    _, rep = orc.cg_ir(A, b, half_band=k, inner_tol=1e-12, max_inner=5000, max_outer=400)
    if rho > 1.05:
        assert rep.status == 3
        return
    assert rho <= 0.8, "case outside the pinned range"
    assert rep.status == 0
    if eq4 < 1.0:
        assert rep.status == 0
    predicted = 1.0 + np.log(1e14) / np.log(1.0 / rho)
    assert 0.75 * predicted <= rep.iters_high <= 1.25 * predicted, (rep.iters_high, predicted)


def test_converged_start_takes_one_confirming_phase(orc):
    # x0 = the binary64 solution: its backward error is already at rounding
    # level, but only a correction shows that x is accurate -- one inner
    # phase from a rounding-level residual moves x by about u cond, and the
    # stopping rule accepts after that residual
    A = spdgen.covariance(300, 2)
    rng = np.random.Generator(np.random.PCG64(5))
    Xt = rng.standard_normal((1, 300))
    B = spdgen.accurate_product(A, Xt)
    X0, _ = orc.solve(A, B)
    X, rep = orc.cg_ir(A, B, X0t=X0, half_band=-1)
    assert rep.status == 0 and rep.iters_high == 2 and rep.iters_low >= 1
    assert np.abs(X - Xt).max() / np.abs(Xt).max() <= 1e-13


def test_cg_success_implies_forward_error_bar(orc):
    # Algorithm 2 with a banded operator contracts by a fixed factor per
    # outer step; eta <= tol alone stops it while x still carries about
    # cond * tol of error.  With the stopping rule, success means the
    # forward error meets 10 cond u against x_true
    n, d, k = 600, 1, 16
    A = spdgen.covariance(n, d)
    lam = np.linalg.eigvalsh(A)
    cond = lam[-1] / lam[0]
    rng = np.random.Generator(np.random.PCG64(6))
    Xt = rng.standard_normal((2, n))
    B = spdgen.accurate_product(A, Xt)
    X, rep = orc.cg_ir(A, B, half_band=k)
    assert rep.status == 0
    for c in range(2):
        assert np.abs(X[c] - Xt[c]).max() / np.abs(Xt[c]).max() <= 10 * cond * U64
