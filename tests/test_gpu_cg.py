"""GPU parity of Algorithm 2 (CG with iterative refinement, Section 3.2) on
the dense and banded binary32 operators (Section 4) against the oracle
(oracle.cg_ir, pinned on the CPU).

* Steps: after k <= 3 products (one phase, x0 = 0) X agrees with the
  oracle's to 4 k n u32 of max|x| (the two sum the binary32 dot products in
  different orders); from k = 2 on X depends on every entry of the product.
* Whole runs at sizes spanning several workgroups with ragged tails, the
  VALU (1-4 right-hand sides) and MFMA (5-32 per block, and two blocks)
  products and the band kernel: status as the oracle's, residual count
  within +-1, products within +-max(3, 10 %), eta <= 1e-14 recomputed by
  the oracle and the forward error inside the normwise bound
  2 (eta + u) kappa_inf(A).
* The paper's size, n = 70000 with d in {1, 2, 4}: eta <= 1e-14 and the
  2-norm error bound ||x - x_true||_2 <= (||r||_2 + u ||b||_2) / lambda_min
  with lambda_min bounded in closed form (spdgen.covariance_cond_bound).
"""
import math
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24
ETA = {1: math.log(2.0), 2: math.pi ** 2 / 12.0, 4: 7.0 * math.pi ** 4 / 720.0}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_cg(spd, A, Bt, band, **kw):
    import torch
    H = spd.cg_prepare(dev(A), half_band=band)
    X, rep = spd.cg_refine(H, dev(A), dev(Bt), opts=spd.cg_default_opts(**kw))
    torch.cuda.synchronize()
    H.close()
    return X.cpu().numpy(), rep


@pytest.mark.parametrize("band", [-1, 3])
@pytest.mark.parametrize("m", [1, 6])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_cg_steps_match_oracle(spd, orc, band, m, k):
    n = 777
    _say(f"cg steps n={n} band={band} m={m} k={k}")
    A = spdgen.covariance(n, 1)
    Bt = spdgen.rhs(n, m, 100 + m)
    X, rep = _gpu_cg(spd, A, Bt, band, max_outer=1, max_inner=k, inner_tol=0.0)
    Xo, ro = orc.cg_ir(A, Bt, half_band=band, max_outer=1, max_inner=k, inner_tol=0.0)
    assert (rep.iters_low, rep.iters_high) == (ro.iters_low, ro.iters_high) == (k, 2)
    err = np.abs(X - Xo).max(axis=1) / np.abs(Xo).max(axis=1)
    assert err.max() <= 4 * k * n * U32, err.max()


CASES = [
    (300, 1, -1, 1), (777, 2, -1, 3), (777, 4, -1, 8), (1000, 1, -1, 33),
    (777, 1, 16, 1), (1000, 2, 16, 5), (777, 4, 2, 4), (300, 1, 0, 2),
]


@pytest.mark.parametrize("n,d,band,m", CASES)
def test_cg_ir_matches_oracle(spd, orc, n, d, band, m):
    _say(f"cg-ir n={n} d={d} band={band} m={m}")
    A = spdgen.covariance(n, d)
    Xt = spdgen.rhs(n, m, 7 * n + d)
    Bt = spdgen.accurate_product(A, Xt)
    X, rep = _gpu_cg(spd, A, Bt, band)
    Xo, ro = orc.cg_ir(A, Bt, half_band=band)
    _say(f"  library {rep.status} {rep.iters_low}/{rep.iters_high} eta {rep.eta:.2e}; "
         f"oracle {ro.status} {ro.iters_low}/{ro.iters_high}")
    assert rep.status == ro.status
    assert abs(rep.iters_high - ro.iters_high) <= 1
    assert abs(rep.iters_low - ro.iters_low) <= max(3, 0.1 * ro.iters_low)
    if ro.status == 0:
        eta = orc.backward_error(A, X, Bt).max()
        assert eta <= 1e-14
        kinf = np.abs(A).sum(axis=1).max() * np.abs(np.linalg.inv(A)).sum(axis=1).max()
        fe = (np.abs(X - Xt).max(axis=1) / np.abs(Xt).max(axis=1)).max()
        assert fe <= 2 * (eta + U64) * kinf


def test_cg_band_violating_eq4_reports_divergence(spd, orc):
    n, a = 300, 0.01
    A = np.asfortranarray((1 - a) * np.eye(n) + a * np.ones((n, n)))
    Bt = spdgen.rhs(n, 2, 3)
    X, rep = _gpu_cg(spd, A, Bt, 0)
    _, ro = orc.cg_ir(A, Bt, half_band=0)
    assert rep.status == spd.ERR_NO_CONVERGENCE and ro.status == 3


def test_cg_zero_rhs_and_warm_start(spd, orc):
    import torch
    n = 500
    A = spdgen.covariance(n, 2)
    X, rep = _gpu_cg(spd, A, np.zeros((2, n)), -1)
    assert rep.status == 0 and rep.iters_low == 0 and rep.iters_high == 1 and not X.any()
    # a converged start takes one confirming phase (the stopping rule needs a
    # correction), like the oracle's
    Xt = spdgen.rhs(n, 1, 9)
    Bt = spdgen.accurate_product(A, Xt)
    H = spd.cg_prepare(dev(A))
    Xd = dev(Xt.copy())
    _, rep = spd.cg_refine(H, dev(A), dev(Bt), Xd)
    torch.cuda.synchronize()
    _, ro = orc.cg_ir(A, Bt, X0t=Xt.copy(), half_band=-1)
    assert rep.status == 0 and ro.status == 0
    assert rep.iters_high == ro.iters_high == 2 and rep.iters_low >= 1


@pytest.mark.parametrize("d", [1, 2, 4])
@pytest.mark.parametrize("band,m", [(-1, 1), (-1, 32), (16, 1), (16, 32)])
def test_cg_covariance_n70000(spd, d, band, m):
    import torch
    n = 70000
    _say(f"cg covariance n={n} d={d} band={band} m={m}")
    A = spdgen.covariance(n, d, backend="torch", device="cuda")
    _, sx = spdgen.seeds(5, d)
    Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    H = spd.cg_prepare(A, half_band=band)
    X, rep = spd.cg_refine(H, A, B)
    torch.cuda.synchronize()
    H.close()
    R, eta = spd.residual(A, X, B)
    lam_min = 2.0 - 2.0 * ETA[d]
    err = (X - Xt).norm(dim=1)
    bound = (R.norm(dim=1) + U64 * B.norm(dim=1)) / lam_min
    _say(f"  status {rep.status} iters {rep.iters_low}/{rep.iters_high} eta {rep.eta:.2e} "
         f"err/bound {float((err / bound).max()):.2f}")
    assert rep.status == 0
    assert rep.eta <= 1e-14 and float(eta.max()) <= 1e-14
    assert bool((err <= bound).all())
    del A, B, X, Xt, R
    torch.cuda.empty_cache()


def test_cg_handle_reuse_is_bitwise_equal(spd):
    """One handle re-prepared dense -> band -> dense (the operator buffer and
    workspace are reused or rebuilt) gives exactly the results of fresh
    handles: every reduction is in a fixed order."""
    import torch
    n, m = 900, 3
    A = dev(spdgen.covariance(n, 2))
    Bt = dev(spdgen.rhs(n, m, 31))
    fresh = {}
    for band in (-1, 8):
        H = spd.cg_prepare(A, half_band=band)
        fresh[band] = spd.cg_refine(H, A, Bt)[0].clone()
        H.close()
    H = spd.CG()
    for band in (-1, 8, -1):
        spd.cg_prepare(A, half_band=band, H=H)
        X, rep = spd.cg_refine(H, A, Bt)
        torch.cuda.synchronize()
        assert rep.status == 0
        assert torch.equal(X, fresh[band])
    H.close()


@pytest.mark.parametrize("m", [1, 3])
def test_cg_band_graph_matches_direct_launches(spd, m):
    """Banded iterations are replayed from a captured graph (about a hundred
    replays per solve, with host checks between them); with kernel profiling
    on, the same iterations are launched one by one.  Both give the same bits."""
    import torch
    n = 3000
    A = dev(spdgen.covariance(n, 1))
    Bt = dev(spdgen.rhs(n, m, 41))
    H = spd.cg_prepare(A, half_band=16)
    X1, r1 = spd.cg_refine(H, A, Bt)
    torch.cuda.synchronize()
    spd.profile_enable(True)
    try:
        X2, r2 = spd.cg_refine(H, A, Bt)
        torch.cuda.synchronize()
    finally:
        spd.profile_enable(False)
    H.close()
    assert r1.status == r2.status == 0
    assert (r1.iters_low, r1.iters_high) == (r2.iters_low, r2.iters_high) and r1.iters_low > 100
    assert torch.equal(X1, X2)


@pytest.mark.parametrize("n", [1, 2, 33])
@pytest.mark.parametrize("band", [-1, 0, 1])
@pytest.mark.parametrize("m", [1, 5])
def test_cg_tiny_systems_match_oracle(spd, orc, n, band, m):
    """Sizes below one 256-row tile (padding everywhere; empty k-slices for
    some waves of the split product): status and counts as the oracle's."""
    A = spdgen.covariance(n, 1)
    Bt = spdgen.rhs(n, m, 50 + n)
    X, rep = _gpu_cg(spd, A, Bt, band)
    Xo, ro = orc.cg_ir(A, Bt, half_band=band)
    assert rep.status == ro.status
    assert abs(rep.iters_high - ro.iters_high) <= 1
    assert abs(rep.iters_low - ro.iters_low) <= max(3, 0.1 * ro.iters_low)
    if ro.status == 0:
        assert orc.backward_error(A, X, Bt).max() <= 1e-14
