"""GPU parity of the BF16 / FP16 factor modes (Algorithm 1 with the trailing
update's operands rounded to bfloat16 / binary16, binary32 accumulation,
after diagonal equilibration and, for FP16, the power-of-two scale mu) and
of the fallback chain BF16/FP16 -> FP32 -> FP64, against the oracle's
emulation of the same algorithm.

Bars:
  * outcome (precision finally used, number of fallbacks): the oracle's;
  * iteration counts: at most the oracle's + 1.  The library rounds only the
    operands of the updates that cross 128-wide panels (the diagonal blocks
    and panel solves stay binary32); the oracle rounds every update product.
    The library's factor is therefore at least as accurate and may need fewer
    corrections -- many fewer when n is a few panels wide;
  * refined solutions: eta <= 1e-14 recomputed by the oracle and forward error
    <= 10 cond(A) 2^-53 against X_true and the oracle's binary64 solution;
  * factor of H = mu D A D (binary32, rounded): componentwise backward bound
    |H - L L^T| <= (2 u_h + u_h^2 + 4 (n+1) u32) |L||L^T| (each product of
    rounded operands is off by at most 2 u_h + u_h^2 relatively);
  * breakdown column without fallback: exactly the oracle's.
"""
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24
UH = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
PREC_ID = {"bf16": 0, "fp16": 1, "fp32": 2, "fp64": 3}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def fwd_err(X, Xref):
    X, Xref = np.atleast_2d(X), np.atleast_2d(Xref)
    return np.max(np.abs(X - Xref), axis=1) / np.max(np.abs(Xref), axis=1)


def iters_close(gpu, orc):
    return gpu <= orc + 1


# (n, cond, m, prec): converging cases in both formats, the BF16 -> FP32
# fallback at cond 1e3 and the FP16 -> FP32 fallback at cond 1e5 (the outcomes
# the analysis of Eq. (4) predicts: cond * u_h well below / above 1).
# Sizes past 2048 take the group trailing update on 256 x 256 tiles (three
# groups of 1024 columns at n = 3000, ragged last group at 2300).
CASES = [(1024, 1e1, 1, "bf16"), (1024, 1e1, 1, "fp16"), (700, 1e2, 2, "fp16"), (1024, 1e3, 1, "fp16"),
         (1024, 1e3, 1, "bf16"), (1300, 1e5, 1, "fp16"), (512, 1e5, 3, "bf16"), (257, 1e1, 1, "fp16"),
         (129, 1e2, 4, "bf16"), (3000, 1e2, 2, "fp16"), (2300, 1e1, 1, "bf16"), (3000, 1e3, 1, "fp16")]


@pytest.mark.parametrize("n,cond,m,prec", CASES)
def test_posv_half_matches_oracle(spd, orc, n, cond, m, prec):
    _say(f"posv {prec} n={n} cond={cond} m={m}")
    s = spdgen.system(n, cond, m, config=2, index=n + 3 * m)
    X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec=prec)
    Xh = host(X)
    F.close()
    _, orep = orc.ir(s.A, s.Bt, prec=prec)
    _say("  gpu", rep.as_dict(), "oracle", orep)
    assert rep.status == 0, rep.as_dict()
    assert orep.status == 0
    assert rep.prec_used == orep.prec_used and rep.fallbacks == orep.fallbacks, (rep.as_dict(), orep)
    assert iters_close(rep.iters_low, orep.iters_low), (rep.as_dict(), orep)
    eta = orc.backward_error(s.A, Xh, s.Bt)
    assert np.all(eta <= 1e-14), eta
    bound = 10 * cond * U64
    Xo, info = orc.solve(s.A, s.Bt)
    assert info == 0
    assert np.all(fwd_err(Xh, Xo) <= bound), (fwd_err(Xh, Xo), bound)
    assert np.all(fwd_err(Xh, s.Xt) <= bound), (fwd_err(Xh, s.Xt), bound)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("n,cond", [(640, 1e1), (1100, 1e2), (3000, 1e2), (4400, 1e1)])
def test_factor_half_backward_bound(spd, orc, prec, n, cond):
    _say(f"factor {prec} n={n} cond={cond}")
    A = spdgen.logspaced(n, cond, 300 + n)
    F, info, st = spd.factor(dev(A), prec)
    assert info == 0 and st == 0
    L, d, mu = spd.export(F)
    L, d = host(L), host(d)
    F.close()
    dref = 1.0 / np.sqrt(np.diag(A))
    assert np.array_equal(d, dref)
    if prec == "fp16":
        # largest power of two <= 0.1 * 65504
        assert mu == 4096.0
    else:
        assert mu == 1.0
    H = (((dref[:, None] * A) * dref[None, :]) * mu).astype(np.float32).astype(np.float64)
    assert np.count_nonzero(np.triu(L, 1)) == 0
    assert np.all(np.diag(L) > 0)
    absLL = np.abs(L) @ np.abs(L.T)
    E = np.abs(H - L @ L.T)
    uh = UH[prec]
    c = 2 * uh + uh * uh + 4 * (n + 1) * U32
    ratio = np.max(E / absLL)
    _say("  max |H - LL^T| / (|L||L^T|) =", ratio, "bound", c)
    assert np.all(E <= c * absLL), ratio
    # the operands really were rounded: the binary32 factor of the same
    # matrix is much closer to its H (rules out a silent binary32 update)
    F32, info, _ = spd.factor(dev(A), "fp32")
    L32 = host(spd.export(F32)[0])
    F32.close()
    H32 = ((dref[:, None] * A) * dref[None, :]).astype(np.float32).astype(np.float64)
    ratio32 = np.max(np.abs(H32 - L32 @ L32.T) / (np.abs(L32) @ np.abs(L32.T)))
    _say("  binary32 factor ratio", ratio32)
    assert ratio > 16 * ratio32


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("n,j0", [(400, 1), (400, 129), (400, 256), (600, 385)])
def test_breakdown_column_half(spd, orc, prec, n, j0):
    _say(f"breakdown {prec} n={n} j0={j0}")
    A = spdgen.indefinite(n, j0, seed=j0 + 5)
    F, info, st = spd.factor(dev(A), prec)
    F.close()
    B = np.ones((1, n))
    _, orep = orc.ir(A, B, prec=prec, fallback=False)
    assert orep.info == j0
    assert st == 2 and info == j0, (st, info)


def test_half_breakdown_falls_back(spd, orc):
    # an indefinite matrix: every precision breaks down, posv ends at FP64 with NOT_SPD
    n, j0 = 300, 200
    A = spdgen.indefinite(n, j0, seed=3)
    B = np.ones((1, n))
    X, rep, F = spd.posv(dev(A), dev(B), prec="bf16")
    F.close()
    assert rep.status == 2 and rep.prec_used == 3 and rep.info == j0
    assert rep.fallbacks == 2


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_half_breakdown_then_binary32_succeeds(spd, orc, prec):
    # SPD, with rows 0 and 128 coupled by 1 - 1e-4 (eigenvalues 2 - 1e-4 and
    # 1e-4 in that plane).  The second panel's pivot is 1 - l^2 with
    # l = 1 - 1e-4 from the first panel: rounded to binary16 or bfloat16 as an
    # update operand, l becomes exactly 1 and the pivot 0 (a breakdown at
    # column 129); binary32 keeps l and a pivot of about 2e-4.  spd_posv reads
    # the factorisation's outcome only with the first residual, so this checks
    # that a half-precision breakdown found there still restarts at binary32
    # and ends with a correct solution.
    n, j = 300, 128
    A = np.eye(n)
    A[0, j] = A[j, 0] = 1.0 - 1e-4
    F, info, st = spd.factor(dev(A), prec)
    F.close()
    assert st == 2 and info == j + 1, (st, info)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((2, n))
    X, rep, F = spd.posv(dev(A), dev(B), prec=prec)
    F.close()
    assert rep.status == 0 and rep.prec_used == PREC_ID["fp32"] and rep.fallbacks == 1, rep.as_dict()
    assert np.all(orc.backward_error(A, host(X), B) <= 1e-14)
    Xo, oinfo = orc.solve(A, B)
    assert oinfo == 0
    cond = (2.0 - 1e-4) / 1e-4
    fe = np.max(np.abs(host(X) - Xo)) / np.max(np.abs(Xo))
    assert fe <= 10 * cond * 2.0 ** -53, fe


def test_half_switch_precision_on_one_handle(spd, orc):
    # the same handle factors at FP16, then FP32, then BF16; every solve is correct
    n, cond = 500, 1e2
    s = spdgen.system(n, cond, 1, config=2, index=77)
    F = None
    for prec in ("fp16", "fp32", "bf16", "fp16"):
        X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec=prec, F=F)
        assert rep.status == 0 and rep.prec_used == PREC_ID[prec]
        assert np.all(orc.backward_error(s.A, host(X), s.Bt) <= 1e-14)
    F.close()
