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
