"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (each derived from the arithmetic it bounds):
  * refined solutions: backward error eta <= 1e-14 recomputed by the oracle,
    and normwise forward error <= 10 cond(A) 2^-53 against the oracle's binary64
    solution and against X_true (B formed in double-double);
  * factor L of H: componentwise backward bound |H - L L^T| <= c (n+1) u |L||L^T|
    with c = 4, and distance to the oracle's factor <= n u cond(H) ||L||;
  * residual kernel: |R - R_oracle| <= (n+1) u64 (|A||X| + |B|) elementwise;
  * breakdown column (an integer): exactly the oracle's.
"""
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


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


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,cond,m", [(1024, 1e4, 1), (700, 1e2, 3), (1300, 1e6, 2), (257, 1e4, 1),
                                      (64, 1e3, 1), (512, 1e5, 8)])
def test_posv_fp32_refined_matches_oracle(spd, orc, n, cond, m):
    _say(f"posv fp32 n={n} cond={cond} m={m}")
    s = spdgen.system(n, cond, m, config=0, index=n + m)
    X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec="fp32")
    Xh = host(X)
    F.close()
    assert rep.status == 0, rep.as_dict()
    assert rep.prec_used == 2 and rep.fallbacks == 0
    eta = orc.backward_error(s.A, Xh, s.Bt)
    assert np.all(eta <= 1e-14), eta
    Xo, info = orc.solve(s.A, s.Bt)
    assert info == 0
    bound = 10 * cond * U64
    assert np.all(fwd_err(Xh, Xo) <= bound), (fwd_err(Xh, Xo), bound)
    assert np.all(fwd_err(Xh, s.Xt) <= bound), (fwd_err(Xh, s.Xt), bound)
    # iteration counts agree with the oracle's emulation of Algorithm 1 (+-1)
    _, orep = orc.ir(s.A, s.Bt, prec="fp32")
    assert abs(rep.iters_low - orep.iters_low) <= 1, (rep.as_dict(), orep)
    _say("  iters", rep.iters_low, rep.iters_high, "eta", rep.eta, "oracle iters", orep.iters_low)


@pytest.mark.parametrize("n,cond,m", [(1024, 1e4, 1), (333, 1e6, 2)])
def test_posv_fp64_one_step(spd, orc, n, cond, m):
    _say(f"posv fp64 n={n} cond={cond} m={m}")
    s = spdgen.system(n, cond, m, config=0, index=7 + n)
    X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec="fp64")
    Xh = host(X)
    F.close()
    assert rep.status == 0 and rep.prec_used == 3
    assert (rep.iters_low, rep.iters_high) == (1, 1)
    Xo, _ = orc.solve(s.A, s.Bt)
    assert np.all(fwd_err(Xh, Xo) <= 10 * cond * U64)
    assert np.all(orc.backward_error(s.A, Xh, s.Bt) <= 1e-14)


@pytest.mark.parametrize("n,cond", [(300, 1e3), (1024, 1e4), (777, 1e2)])
def test_factor_fp32_against_oracle(spd, orc, n, cond):
    _say(f"factor fp32 n={n}")
    A = spdgen.logspaced(n, cond, 100 + n)
    F, info, st = spd.factor(dev(A), "fp32")
    assert info == 0 and st == 0
    L, d, mu = spd.export(F)
    L, d = host(L), host(d)
    F.close()
    # equilibration is the plain definition, bit for bit
    dref = 1.0 / np.sqrt(np.diag(A))
    assert np.array_equal(d, dref)
    assert mu == 1.0
    H = ((dref[:, None] * A) * dref[None, :]).astype(np.float32).astype(np.float64)
    assert np.count_nonzero(np.triu(L, 1)) == 0
    absLL = np.abs(L) @ np.abs(L.T)
    E = np.abs(H - L @ L.T)
    assert np.all(E <= 4 * (n + 1) * U32 * absLL), np.max(E / absLL)
    Lref, info = orc.potrf(H)
    assert info == 0
    lam = np.linalg.eigvalsh(H)
    condH = lam[-1] / lam[0]
    dist = np.max(np.abs(L - Lref)) / np.max(np.abs(Lref))
    _say("  factor dist", dist, "bound", n * U32 * condH)
    assert dist <= n * U32 * condH


@pytest.mark.parametrize("n,cond", [(300, 1e3), (1024, 1e4)])
def test_factor_fp64_against_oracle(spd, orc, n, cond):
    _say(f"factor fp64 n={n}")
    A = spdgen.logspaced(n, cond, 200 + n)
    F, info, st = spd.factor(dev(A), "fp64")
    assert info == 0
    L, d, mu = spd.export(F)
    L = host(L)
    F.close()
    E = np.abs(A - L @ L.T)
    absLL = np.abs(L) @ np.abs(L.T)
    assert np.all(E <= 4 * (n + 1) * U64 * absLL), np.max(E / absLL)
    Lref, _ = orc.potrf(A)
    dist = np.max(np.abs(L - Lref)) / np.max(np.abs(Lref))
    _say("  factor dist", dist)
    assert dist <= n * U64 * cond


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,j0", [(400, 1), (400, 100), (400, 256), (400, 257), (400, 400), (600, 513)])
def test_breakdown_column_matches_oracle(spd, orc, prec, n, j0):
    _say(f"breakdown {prec} n={n} j0={j0}")
    A = spdgen.indefinite(n, j0, seed=j0)
    _, oinfo = orc.potrf(A)
    assert oinfo == j0
    F, info, st = spd.factor(dev(A), prec)
    F.close()
    assert st == spd.ERR_NOT_SPD
    assert info == oinfo


@pytest.mark.parametrize("n,m", [(1000, 1), (777, 5), (300, 64), (130, 70), (2049, 1), (513, 2), (65, 1), (1, 1),
                                 (1100, 3), (1000, 12), (700, 32), (129, 17)])
def test_residual_kernel_elementwise(spd, orc, n, m):
    _say(f"residual n={n} m={m}")
    s = spdgen.system(n, 1e3, m, config=1, index=n)
    rng = np.random.Generator(np.random.PCG64(n))
    X = s.Xt + 1e-6 * rng.standard_normal(s.Xt.shape)
    R, eta = spd.residual(dev(s.A), dev(X), dev(s.Bt))
    R = host(R)
    Ro = orc.residual(s.A, X, s.Bt)
    bound = (n + 1) * U64 * ((np.abs(X) @ np.abs(s.A)) + np.abs(s.Bt))
    assert np.all(np.abs(R - Ro) <= bound)
    eo = orc.backward_error(s.A, X, s.Bt)
    np.testing.assert_allclose(eta, eo, rtol=1e-6)


def test_golden_tiny_systems(spd, orc):
    import json
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "exact_small.json")
    for c in json.load(open(path))["cases"]:
        n = c["n"]
        A = np.array(c["A"], dtype=np.float64)
        b = np.array(c["b"], dtype=np.float64)
        _say(f"golden n={n}")
        X, rep, F = spd.posv(dev(A), dev(b), prec="fp32")
        F.close()
        xe = np.array([float(Fraction(v)) for v in c["x"]])
        cond = np.linalg.cond(A)
        assert rep.status == 0
        assert np.max(np.abs(host(X) - xe)) <= 10 * cond * U64 * np.max(np.abs(xe))


def test_hilbert_falls_back_to_fp64(spd, orc):
    n = 10
    A = spdgen.hilbert(n)
    b = A @ np.ones(n)
    X, rep, F = spd.posv(dev(A), dev(b), prec="fp32")
    F.close()
    _, orep = orc.ir(A, b, prec="fp32")
    assert rep.status == 0 and rep.prec_used == 3 and rep.fallbacks >= 1
    assert orep.prec_used == 3


def test_nan_rhs_reports_no_convergence(spd):
    s = spdgen.system(300, 1e2, 1, config=0, index=5)
    B = s.Bt.copy()
    B[0, 17] = np.nan
    X, rep, F = spd.posv(dev(s.A), dev(B), prec="fp32", opts=spd.default_opts(fallback=0))
    F.close()
    assert rep.status == spd.ERR_NO_CONVERGENCE
    assert np.isnan(rep.eta)


def test_max_iter_zero(spd, orc):
    s = spdgen.system(500, 1e4, 1, config=0, index=6)
    X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec="fp32", opts=spd.default_opts(max_iter=0, fallback=0))
    F.close()
    assert (rep.iters_low, rep.iters_high) == (1, 1)
    assert rep.status == spd.ERR_NO_CONVERGENCE


def test_edge_sizes(spd, orc):
    import torch
    # n = 1
    A = np.array([[4.0]])
    X, rep, F = spd.posv(dev(A), dev(np.array([2.0])), prec="fp32")
    F.close()
    assert rep.status == 0 and abs(host(X)[0] - 0.5) <= 4 * U64
    # n = 0
    A0 = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    B0 = torch.zeros((0,), dtype=torch.float64, device="cuda")
    X, rep, F = spd.posv(A0, B0, prec="fp32")
    F.close()
    assert rep.status == 0
    # ragged: n = NB + 1 and NB - 1
    for n in (255, 257, 513):
        s = spdgen.system(n, 1e3, 2, config=0, index=900 + n)
        X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec="fp32")
        F.close()
        assert rep.status == 0
        assert np.all(orc.backward_error(s.A, host(X), s.Bt) <= 1e-14)


def test_only_lower_triangle_read(spd, orc):
    import torch
    n = 300
    s = spdgen.system(n, 1e3, 1, config=0, index=8)
    # a row-major contiguous tensor T is read as the column-major matrix whose
    # element (i, j) sits at T[j][i]; the library may only read i >= j, i.e. the
    # upper triangle of T.  Poison T's strict lower triangle.
    T = dev(s.A)
    r, c = torch.tril_indices(n, n, -1, device="cuda")
    T[r, c] = float("nan")
    X, rep, F = spd.posv(T, dev(s.Bt), prec="fp32")
    F.close()
    assert rep.status == 0
    assert np.all(orc.backward_error(s.A, host(X), s.Bt) <= 1e-14)


def test_deterministic(spd):
    s = spdgen.system(900, 1e4, 3, config=0, index=9)
    A, B = dev(s.A), dev(s.Bt)
    X1, r1, F1 = spd.posv(A, B, prec="fp32")
    X2, r2, F2 = spd.posv(A, B, prec="fp32", F=F1)  # handle reuse
    assert np.array_equal(host(X1), host(X2))
    assert r1.iters_low == r2.iters_low
    F1.close()


def test_separate_calls_match_posv(spd, orc):
    s = spdgen.system(600, 1e4, 2, config=0, index=10)
    A, B = dev(s.A), dev(s.Bt)
    F, info, st = spd.factor(A, "fp32")
    X0 = spd.solve(F, B)
    x0 = host(X0).copy()
    # the first solve alone: a binary32-accurate solution
    Xo, _ = orc.solve(s.A, s.Bt)
    assert np.all(fwd_err(x0, Xo) <= 600 * U32 * 1e4)
    rep = spd.refine(F, A, B, X0)
    assert rep.status == 0
    Xp, rep2, F2 = spd.posv(A, B, prec="fp32")
    assert np.array_equal(host(X0), host(Xp))
    F.close()
    F2.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,m", [(640, 11), (400, 64), (1100, 3)])
def test_posv_many_rhs(spd, orc, prec, n, m):
    _say(f"posv {prec} n={n} m={m}")
    cond = 1e3
    s = spdgen.system(n, cond, m, config=0, index=3000 + n + m)
    X, rep, F = spd.posv(dev(s.A), dev(s.Bt), prec=prec)
    Xh = host(X)
    F.close()
    assert rep.status == 0, rep.as_dict()
    assert np.all(orc.backward_error(s.A, Xh, s.Bt) <= 1e-14)
    Xo, _ = orc.solve(s.A, s.Bt)
    assert np.all(fwd_err(Xh, Xo) <= 10 * cond * U64)


def test_solve_only_first_step_accuracy(spd, orc):
    # Algorithm 1's first solve alone with a binary64 factor: already binary64-accurate
    s = spdgen.system(777, 1e4, 4, config=0, index=4000)
    F, info, st = spd.factor(dev(s.A), "fp64")
    X = host(spd.solve(F, dev(s.Bt)))
    F.close()
    Xo, _ = orc.solve(s.A, s.Bt)
    assert np.all(fwd_err(X, Xo) <= 10 * 1e4 * U64)
