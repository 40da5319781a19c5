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


def test_ir_factor_exact_factor_one_step(orc):
    # the binary64 factor itself: one solve already reaches the binary64 floor
    A, Xt, B = _ir_factor_case()
    L, info = orc.potrf(A)
    assert info == 0
    X, rep = orc.ir_factor(A, L, B, prec="fp64")
    assert rep.status == 0 and (rep.iters_low, rep.iters_high) == (1, 1)
    assert rep.eta <= 2.0 ** -51


@pytest.mark.parametrize("alpha", [0.9, 1.1, 1.25])
def test_ir_factor_scaled_factor_closed_form(orc, alpha):
    # L~ = alpha L gives L~ L~^T = alpha^2 A, so with c = 1 - 1/alpha^2 the
    # error after j solves is exactly -c^j x: x_j = (1 - c^j) x and the j-th
    # residual is r_j = c^j b, so
    #   eta_j = |c|^j ||b|| / (||A|| ||x|| |1 - c^j| + ||b||),
    # and the loop stops at the first eta_j <= 2^-51 (Eq. (4):
    # ||A^{-1} dA|| = |1 - alpha^2| < 1 here).
    A, Xt, B = _ir_factor_case()
    L, _ = orc.potrf(A)
    X, rep = orc.ir_factor(A, alpha * L, B, prec="fp64", max_iter=200)
    c = 1.0 - 1.0 / alpha ** 2
    an = np.abs(A).sum(axis=1).max()
    nb, nx = np.abs(B).max(), np.abs(Xt).max()
    j = 1
    while abs(c) ** j * nb / (an * nx * abs(1.0 - c ** j) + nb) > 2.0 ** -51:
        j += 1
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
    refinement of line 1's own binary32 factor without equilibration."""
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
