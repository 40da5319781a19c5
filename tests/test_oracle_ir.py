"""Pins for the oracle's emulation of Algorithm 1 (Cholesky with iterative refinement)."""
import numpy as np
import pytest

import spdgen

U64 = 2.0 ** -53


def test_fp64_factor_converges_without_corrections(orc):
    # special case: a binary64 factor is already backward stable -> "1 / 1"
    s = spdgen.system(300, 1e4, 2, config=0, index=1)
    X, rep = orc.ir(s.A, s.Bt, prec="fp64")
    assert rep.status == 0 and rep.prec_used == 3
    assert (rep.iters_low, rep.iters_high) == (1, 1)
    Xd, _ = orc.solve(s.A, s.Bt)
    assert np.array_equal(X, Xd)


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_fp32_refinement_reaches_fp64_accuracy(orc, cond):
    n = 256
    s = spdgen.system(n, cond, 1, config=0, index=2)
    X, rep = orc.ir(s.A, s.Bt, prec="fp32")
    assert rep.status == 0 and rep.prec_used == 2 and rep.fallbacks == 0
    assert rep.eta <= 1e-14
    # contraction ~ cond * u32 per step: a handful of corrections at most
    assert 2 <= rep.iters_low <= 6
    fwd = np.max(np.abs(X - s.Xt)) / np.max(np.abs(s.Xt))
    assert fwd <= 10 * cond * U64
    assert np.all(orc.backward_error(s.A, X, s.Bt) <= 1e-14)


def test_half_precision_operands_small_cond(orc):
    s = spdgen.system(128, 10.0, 1, config=2, index=0)
    for p in ("bf16", "fp16"):
        X, rep = orc.ir(s.A, s.Bt, prec=p)
        assert rep.status == 0 and rep.fallbacks == 0, (p, rep)
        assert rep.prec_used == orc.PREC[p]
        assert rep.eta <= 1e-14


def test_bf16_falls_back_on_ill_conditioned(orc):
    # cond * u_bf16 = 1e5 * 2^-8 >> 1: refinement cannot converge -> FP32
    s = spdgen.system(128, 1e5, 1, config=2, index=1)
    X, rep = orc.ir(s.A, s.Bt, prec="bf16")
    assert rep.status == 0
    assert rep.fallbacks >= 1 and rep.prec_used in (2, 3)
    assert rep.eta <= 1e-14


def test_hilbert_fp32_falls_back_to_fp64(orc):
    # Hilbert n = 10: cond ~ 1.6e13, far beyond 1/u32; FP32 breaks down or
    # diverges, FP64 (cond * u64 ~ 2e-3 < 1) finishes the job.
    n = 10
    A = spdgen.hilbert(n)
    b = A @ np.ones(n)
    X, rep = orc.ir(A, b, prec="fp32", equilibrate=True)
    assert rep.fallbacks == 1 and rep.prec_used == 3
    assert rep.status == 0


def test_indefinite_is_not_spd_at_every_precision(orc):
    A = spdgen.indefinite(40, 17)
    b = np.ones(40)
    X, rep = orc.ir(A, b, prec="fp32")
    assert rep.status == orc.STATUS_NOT_SPD
    assert rep.info == 17 and rep.prec_used == 3


def test_no_fallback_reports_failure(orc):
    n = 10
    A = spdgen.hilbert(n)
    X, rep = orc.ir(A, A @ np.ones(n), prec="fp32", fallback=False)
    assert rep.status != 0 and rep.prec_used == 2


def test_nan_rhs_terminates(orc):
    s = spdgen.system(64, 1e2, 1, config=0, index=3)
    B = s.Bt.copy()
    B[0, 5] = np.nan
    X, rep = orc.ir(s.A, B, prec="fp32")
    assert rep.status == orc.STATUS_NO_CONVERGENCE
    assert np.isnan(rep.eta)


def test_max_iter_zero(orc):
    s = spdgen.system(64, 1e4, 1, config=0, index=4)
    X, rep = orc.ir(s.A, s.Bt, prec="fp32", max_iter=0, fallback=False)
    assert rep.iters_low == 1 and rep.iters_high == 1
    assert rep.status == orc.STATUS_NO_CONVERGENCE


def test_convergence_condition_eq4(orc):
    # Eq. (4): refinement with inner solves (A + dA) z = r converges when
    # ||A^{-1} dA||_inf < 1.  Build the emulated FP32 factor's dA for a small
    # system and check the prediction matches the observed outcome, on both
    # sides of the threshold (cond 1e3: converges; Hilbert 9: does not).
    def fp32_perturbation(A):
        n = A.shape[0]
        d = 1.0 / np.sqrt(np.diag(A))
        H = (d[:, None] * A * d[None, :]).astype(np.float32)
        L = np.linalg.cholesky(H.astype(np.float64))  # reference only for the norm estimate
        L32 = L.astype(np.float32).astype(np.float64)
        Aeff = (L32 @ L32.T) / d[:, None] / d[None, :]
        return Aeff - A

    for A, should in ((spdgen.logspaced(60, 1e3, 9), True), (spdgen.hilbert(9), False)):
        dA = fp32_perturbation(A)
        q = np.linalg.norm(np.linalg.solve(A, dA), np.inf)
        assert (q < 1) == should, q
        _, rep = orc.ir(A, A @ np.ones(A.shape[0]), prec="fp32", fallback=False)
        assert (rep.status == 0) == should, rep


# --- refinement with a given factor (the perturbed-factor experiment, Fig. 3(b)) ---

def _ir_factor_case(n=200, cond=1e2, seed=31):
    A = spdgen.logspaced(n, cond, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    Xt = rng.standard_normal((1, n))
    B = (A @ Xt[0])[None, :]
    return A, Xt, B


def test_ir_factor_exact_factor_one_correction(orc):
    # the binary64 factor itself, handed in as a given factor: nothing says
    # it is backward stable, so one correction confirms it -- a correction
    # computed from a rounding-level residual, far below the first solve
    A, Xt, B = _ir_factor_case()
    L, info = orc.potrf(A)
    assert info == 0
    X, rep = orc.ir_factor(A, L, B, prec="fp64")
    assert rep.status == 0 and (rep.iters_low, rep.iters_high) == (2, 2)
    assert rep.eta <= 2.0 ** -51
    assert np.abs(X - Xt).max() / np.abs(Xt).max() <= 10 * 1e2 * U64


def _scaled_factor_stop(c, alpha, an, nx, nb, tol=1e-14):
    """The stopping rule applied to the closed-form sequences of the scaled
    factor alpha L (c = 1 - 1/alpha^2): x_j = (1 - c^j) x, r_j = c^j b,
    z_j = c^j x / alpha^2, so with max norms
      eta_j  = |c|^j ||b|| / (||A|| ||x|| |1 - c^j| + ||b||),
      zeta_0 = 1,  zeta_j = |c|^j / (alpha^2 |1 - c^(j+1)|)  (j >= 1).
    Returns the number of residuals at the first k >= 1 where the rule
    accepts x_{k+1}."""
    def eta(j):
        return abs(c) ** j * nb / (an * nx * abs(1.0 - c ** j) + nb)

    def zeta(j):
        return 1.0 if j == 0 else abs(c) ** j / (alpha ** 2 * abs(1.0 - c ** (j + 1)))

    k = 1
    while True:
        if eta(k + 1) <= tol:
            rho = zeta(k) / zeta(k - 1)
            if zeta(k) <= U64:
                return k + 1
            if rho < 0.5 and rho / (1 - rho) * eta(k) <= U64:
                return k + 1
            if rho >= 0.5 and eta(k) <= 2.0 ** -51:
                return k + 1
        k += 1


@pytest.mark.parametrize("alpha", [0.9, 1.1, 1.25])
def test_ir_factor_scaled_factor_closed_form(orc, alpha):
    # L~ = alpha L gives L~ L~^T = alpha^2 A, so the error after j solves is
    # exactly -c^j x with c = 1 - 1/alpha^2 (Eq. (4): ||A^{-1} dA|| =
    # |1 - alpha^2| < 1 here), and both the backward errors and the
    # corrections the stopping rule reads follow in closed form
    A, Xt, B = _ir_factor_case()
    L, _ = orc.potrf(A)
    X, rep = orc.ir_factor(A, alpha * L, B, prec="fp64", max_iter=200)
    c = 1.0 - 1.0 / alpha ** 2
    an = np.abs(A).sum(axis=1).max()
    nb, nx = np.abs(B).max(), np.abs(Xt).max()
    j = _scaled_factor_stop(c, alpha, an, nx, nb)
    assert rep.status == 0
    assert abs(rep.iters_high - j) <= 1, (rep.iters_high, j)
    assert np.abs(X - Xt).max() / np.abs(Xt).max() <= 1e-13


def test_ir_factor_rising_eta_is_taken_for_divergence(orc):
    # alpha = 0.8 (c = -0.5625): the iterate's norm drops from 1.56 ||x|| to
    # 0.68 ||x|| after the first correction, so eta rises once even though
    # the error contracts -- the divergence reading (eta above the first eta)
    # stops it, as it does in the library
    A, Xt, B = _ir_factor_case()
    L, _ = orc.potrf(A)
    X, rep = orc.ir_factor(A, 0.8 * L, B, prec="fp64", max_iter=200)
    assert rep.status == 3 and rep.iters_high == 2


def test_ir_factor_too_large_a_perturbation_diverges(orc):
    # alpha = 0.6: c = 1 - 1/0.36 = -1.78, the error grows every step
    A, Xt, B = _ir_factor_case()
    L, _ = orc.potrf(A)
    X, rep = orc.ir_factor(A, 0.6 * L, B, prec="fp64", max_iter=50)
    assert rep.status == 3


def test_ir_factor_rejects_a_bad_diagonal(orc):
    A, Xt, B = _ir_factor_case(n=50)
    L, _ = orc.potrf(A)
    L = L.copy()
    L[17, 17] = -1.0
    X, rep = orc.ir_factor(A, L, B)
    assert rep.status == 2 and rep.info == 18


def test_ir_factor_fp32_matches_own_factor_when_exact(orc):
    """min(i, j) has the all-ones lower triangle as its Cholesky factor, exact
    in binary32, and the binary32 factorisation reproduces it exactly (every
    pivot is 1, every subtraction exact).  Importing that factor rounded to
    binary32 (Section 3.1, Fig. 3(b) path) must then give bit for bit the
    refinement of the method's own binary32 factor without equilibration."""
    n = 40
    A = spdgen.minij(n)
    L = np.tril(np.ones((n, n)))
    assert np.array_equal(L @ L.T, A)
    b = A @ np.arange(1.0, n + 1.0)
    X1, r1 = orc.ir_factor(A, L, b, prec="fp32", max_iter=30)
    X2, r2 = orc.ir(A, b, prec="fp32", equilibrate=False, fallback=False, max_iter=30)
    assert r1.status == r2.status == 0
    assert (r1.iters_low, r1.iters_high) == (r2.iters_low, r2.iters_high)
    assert np.array_equal(X1, X2)


# --- the stopping rule: success means binary64 accuracy, not only eta <= tol ---

@pytest.mark.parametrize("prec,cond,n", [("fp32", 1e4, 512), ("fp32", 1e6, 512), ("fp16", 1e2, 512),
                                         ("fp16", 1e3, 512), ("fp16", 1e4, 512), ("bf16", 1e1, 512),
                                         ("bf16", 1e1, 1024), ("bf16", 1e2, 512)])
def test_success_implies_forward_error_bar(orc, prec, cond, n):
    # slowly contracting refinements reach eta <= tol (even eta at the
    # binary64 floor) while x still misses the forward-error bar
    # 10 cond u; reported success must mean the bar is met, against both
    # x_true and the binary64 solution.  (Stopping at the first eta <= 2^-51
    # reported success 1.1-4x above the bar for binary16 at cond 1e4 and
    # 1.02x for bfloat16 at cond 10, n = 1024, on these systems.)
    s = spdgen.system(n, cond, 2, config=2, index=11)
    X, rep = orc.ir(s.A, s.Bt, prec=prec, fallback=False)
    if rep.status != 0:
        assert rep.status == orc.STATUS_NO_CONVERGENCE
        return
    bar = 10 * cond * U64
    Xd, _ = orc.solve(s.A, s.Bt)
    for c in range(2):
        scale = np.abs(s.Xt[c]).max()
        assert np.abs(X[c] - s.Xt[c]).max() / scale <= bar, (c, rep)
        assert np.abs(X[c] - Xd[c]).max() / scale <= bar, (c, rep)
    assert np.all(orc.backward_error(s.A, X, s.Bt) <= 1e-14)


def test_success_needs_a_contracting_correction(orc):
    # a low-precision factor is never accepted on its first solve, even
    # when that solve happens to be backward stable to 1e-14: without a
    # correction there is no evidence of the error left (binary32 at cond 10,
    # n = 8: eta after the first solve is about 1e-8 anyway; with tol = 1 the first
    # eta passes the tolerance and one correction is still taken)
    s = spdgen.system(8, 10.0, 1, config=2, index=12)
    X, rep = orc.ir(s.A, s.Bt, prec="fp32", tol=1.0, fallback=False)
    assert rep.status == 0 and rep.iters_high >= 2
    X, rep = orc.ir(s.A, s.Bt, prec="fp64", tol=1.0, fallback=False)
    assert rep.status == 0 and (rep.iters_low, rep.iters_high) == (1, 1)


def test_max_iter_ends_without_success_inside_tol(orc):
    # bfloat16 at cond 1e3 contracts slowly (cond * u_bf16 ~ 4, saved by the
    # scaling): after 3 corrections eta may be small, but the rule has no
    # evidence of binary64 accuracy yet -- no convergence, not success
    s = spdgen.system(256, 1e3, 1, config=2, index=5)
    X, rep = orc.ir(s.A, s.Bt, prec="bf16", max_iter=3, fallback=False)
    assert rep.status == orc.STATUS_NO_CONVERGENCE and rep.iters_low == 4
