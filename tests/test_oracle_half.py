"""Pins for the oracle's binary16 / bfloat16 branch of Algorithm 1's factorisation
(the low-precision factor with half-precision update operands and binary32
accumulation, Section 3.1) and its scaling.

Each pin is chosen so that a plausible mistake in the emulation fails it:
the binary16 operand rounding left out (binary32 operands), bfloat16
rounding used for binary16, or the binary16 scale mu dropped (mu = 1).
Expected values come from closed forms, from hand-expanded 2 x 2 factors
with the rounding done by numpy's / torch's own conversions, and from the
convergence condition of Eq. (4) (cond * u_low below or above one).
"""
import math

import numpy as np
import pytest

import spdgen

U64 = 2.0 ** -53
U16 = 2.0 ** -11   # binary16 unit roundoff
UBF = 2.0 ** -8    # bfloat16 unit roundoff


@pytest.mark.parametrize("theta,mu", [(0.1, 4096.0), (0.05, 2048.0), (1.0, 32768.0), (0.01, 512.0)])
def test_fp16_scale_is_largest_power_of_two_below_theta_xmax(orc, theta, mu):
    # mu = largest power of two <= theta * 65504 (65504 = largest binary16)
    A = spdgen.logspaced(16, 1e2, 3)
    L, d, got, info = orc.lowprec_factor(A, "fp16", theta=theta)
    assert info == 0 and got == mu
    assert mu <= theta * 65504 < 2 * mu
    # equilibrated diagonal is 1, so H_00 = mu and L_00 = sqrt(mu) rounded to binary32
    assert L[0, 0] == float(np.sqrt(np.float32(mu)))


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp64"])
def test_no_scale_outside_fp16(orc, prec):
    A = spdgen.logspaced(16, 1e2, 3)
    _, d, mu, info = orc.lowprec_factor(A, prec)
    assert info == 0 and mu == 1.0
    if prec == "fp64":
        assert np.all(d == 1.0)
    else:
        assert np.array_equal(d, 1.0 / np.sqrt(np.diag(A)))


def _two_by_two(a, fmt):
    """Hand-expanded factorisation on H = mu [[1, a], [a, 1]] (no equilibration):
    l11 = sqrt(h11), l21 = h21 / l11 in binary32, then the update of h22
    with the operand l21 rounded to `fmt` and a binary32 product and
    difference, l22 = sqrt of that.  Rounding by numpy (binary16) or torch
    (bfloat16), not by the oracle."""
    import torch
    mu = 4096.0 if fmt == "fp16" else 1.0
    f32 = np.float32
    h11, h21, h22 = f32(mu), f32(mu * a), f32(mu)
    l11 = np.sqrt(h11)
    l21 = f32(h21 / l11)
    if fmt == "fp16":
        op = f32(np.float16(l21))
    elif fmt == "bf16":
        op = f32(torch.tensor(float(l21), dtype=torch.float32).to(torch.bfloat16).float().item())
    else:
        op = l21
    l22 = np.sqrt(f32(h22 - f32(op * op)))
    return float(l11), float(l21), float(l22)


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_update_operand_rounding_two_by_two(orc, fmt):
    # a = 0.3: l21 = 19.2 (fp16 scale) or 0.3 is inexact in both half
    # formats, and the binary16 and bfloat16 roundings differ, so each
    # format's l22 differs from the other two
    a = 0.3
    A = np.array([[1.0, a], [a, 1.0]])
    L, _, mu, info = orc.lowprec_factor(A, fmt, equilibrate=False)
    assert info == 0
    want = _two_by_two(a, fmt)
    assert (L[0, 0], L[1, 0], L[1, 1]) == want
    others = [_two_by_two(a, f)[2] * math.sqrt((4096.0 if fmt == "fp16" else 1.0) / (4096.0 if f == "fp16" else 1.0))
              for f in ("fp16", "bf16", "fp32") if f != fmt]
    assert all(abs(o - want[2]) > 1e-7 * abs(want[2]) for o in others)


def test_minij_fp16_factor_is_exact(orc):
    # min(i, j) = T T^T with T the all-ones lower triangle; scaled by
    # mu = 4096 the factor is 64 T: every operand (64) is exact in binary16
    # and every update an exact integer in binary32 (mu n <= 2^23)
    n = 1024
    A = spdgen.minij(n)
    L, d, mu, info = orc.lowprec_factor(A, "fp16", equilibrate=False)
    assert info == 0 and mu == 4096.0 and np.all(d == 1.0)
    assert np.array_equal(L, 64.0 * np.tril(np.ones((n, n))))


def test_minij_fp16_solution_exact_after_line_2(orc):
    # with the exact factor and an integer solution (|b| < 2^24), the first solve's
    # binary32 substitutions are exact, so X is x_true and the first
    # residual is exactly zero: one solve, one residual
    n = 1024
    A = spdgen.minij(n)
    rng = np.random.Generator(np.random.PCG64(11))
    xt = rng.integers(-4, 5, size=n).astype(np.float64)
    b = A @ xt
    assert np.abs(b).max() < 2 ** 24
    X, rep = orc.ir(A, b, prec="fp16", equilibrate=False, fallback=False)
    assert rep.status == 0 and rep.prec_used == 1
    assert (rep.iters_low, rep.iters_high) == (1, 1) and rep.eta == 0.0
    assert np.array_equal(X[0], xt)


@pytest.mark.parametrize("n", [128, 256])
def test_fp16_converges_where_bf16_falls_back(orc, n):
    # cond 1e3: cond * u16 = 0.49 < 1 (Eq. (4) can hold), cond * u_bf16 = 3.9 > 1
    cond = 1e3
    s = spdgen.system(n, cond, 1, config=2, index=5)
    X, rep = orc.ir(s.A, s.Bt, prec="fp16")
    assert rep.status == 0 and rep.prec_used == 1 and rep.fallbacks == 0, rep
    assert np.abs(X - s.Xt).max() / np.abs(s.Xt).max() <= 10 * cond * U64
    X, rep = orc.ir(s.A, s.Bt, prec="bf16")
    assert rep.status == 0 and rep.fallbacks == 1 and rep.prec_used == 2, rep


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_half_falls_back_at_cond_1e5(orc, prec):
    # cond 1e5: cond * u16 = 49 and cond * u_bf16 = 390, far above one
    cond = 1e5
    s = spdgen.system(256, cond, 1, config=2, index=5)
    X, rep = orc.ir(s.A, s.Bt, prec=prec)
    assert rep.status == 0 and rep.fallbacks == 1 and rep.prec_used == 2, rep
    assert np.abs(X - s.Xt).max() / np.abs(s.Xt).max() <= 10 * cond * U64


def test_fp16_outcome_does_not_depend_on_theta(orc):
    # mu 4096 (theta 0.1) against 2048 (theta 0.05): powers of two change
    # no rounding of H's significands, only the exponent range, so the
    # outcome is the same and the iterates agree to the refinement's accuracy
    cond = 1e2
    s = spdgen.system(200, cond, 2, config=2, index=6)
    X1, r1 = orc.ir(s.A, s.Bt, prec="fp16", theta=0.1)
    X2, r2 = orc.ir(s.A, s.Bt, prec="fp16", theta=0.05)
    assert r1.status == r2.status == 0 and r1.prec_used == r2.prec_used == 1
    assert abs(r1.iters_low - r2.iters_low) <= 1
    scale = np.abs(s.Xt).max()
    assert np.abs(X1 - X2).max() / scale <= 10 * cond * U64
    for X in (X1, X2):
        assert np.abs(X - s.Xt).max() / scale <= 10 * cond * U64


def test_fp16_factor_error_scale(orc):
    # the half-operand factor's backward error sits near u16 * |L||L^T|,
    # far above binary32's: the ratio separates the formats by orders of
    # magnitude (u16 / u32 = 2^13, u_bf16 / u16 = 2^3)
    A = spdgen.logspaced(96, 1e2, 8)
    res = {}
    for p in ("fp32", "fp16", "bf16"):
        L, d, mu, info = orc.lowprec_factor(A, p)
        H = mu * (d[:, None] * A * d[None, :])
        res[p] = np.abs(H - L @ L.T).max() / np.abs(H).max()
    assert res["fp32"] < 1e-6
    assert 0.1 * U16 < res["fp16"] < 10 * U16
    assert 0.1 * UBF < res["bf16"] < 10 * UBF
