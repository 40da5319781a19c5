"""The paper's model covariance workload (Section 4) on the same path:
a(i,j) = 1/|i-j|^d off the diagonal, 1 + sqrt(i) on it (1-based i), at the
paper's size n = 70000 with m = 32 right-hand sides, d in {1, 2, 4}.

The oracle cannot factor this size in seconds, so the checks are properties
that hold at any size: X_true is drawn by the seeded generator and
B = A X_true is formed in double-double, so the forward error of the
refined binary32 solution is checked against 10 kappa 2^-53 with kappa
bounded in closed form (checked on the CPU against the eigenvalues at
n = 400).

The bound (spdgen.covariance_cond_bound) comes from the symbol of the
Toeplitz part; its derivation is in its docstring.
"""
import math
import sys

import pytest

import spdgen

U64 = 2.0 ** -53
ETA = {1: math.log(2.0), 2: math.pi ** 2 / 12.0, 4: 7.0 * math.pi ** 4 / 720.0}
cond_bound = spdgen.covariance_cond_bound


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("d", [1, 2, 4])
def test_cond_bound_against_eigenvalues(d):
    import numpy as np
    n = 400
    lam = np.linalg.eigvalsh(spdgen.covariance(n, d))
    assert lam[0] >= 2.0 - 2.0 * ETA[d] - 1e-12
    assert lam[-1] / lam[0] <= cond_bound(n, d)


@pytest.mark.gpu
@pytest.mark.parametrize("d", [1, 2, 4])
def test_covariance_n70000_m32(spd, d):
    import torch
    n, m = 70000, 32
    _say(f"covariance n={n} m={m} d={d}")
    A = spdgen.covariance(n, d, backend="torch", device="cuda")
    _, sx = spdgen.seeds(5, d)
    Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    X, rep, F = spd.posv(A, B, prec="fp32")
    torch.cuda.synchronize()
    fe = ((X - Xt).abs().amax(dim=1) / Xt.abs().amax(dim=1)).max().item()
    kappa = cond_bound(n, d)
    _say(f"  status {rep.status} prec {spd.PREC_NAME[rep.prec_used]} iters {rep.iters_low}/{rep.iters_high} "
         f"eta {rep.eta:.2e} fwd {fe:.2e} (bar {10 * kappa * U64:.2e})")
    assert rep.status == 0
    assert spd.PREC_NAME[rep.prec_used] == "fp32" and rep.fallbacks == 0
    assert rep.eta <= 1e-14
    assert fe <= 10 * kappa * U64
    del A, B, X, Xt, F
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("n", [2000, 4096])
@pytest.mark.parametrize("d", [1, 2, 4])
def test_covariance_against_oracle(spd, orc, n, d):
    # the Section 4 matrix at sizes the oracle finishes in seconds: the GPU
    # solution element by element against the oracle's binary64 solve, and
    # the refinement's iteration count against the oracle's emulation of
    # Algorithm 1 (same stopping rule)
    import numpy as np
    import torch
    _say(f"covariance vs oracle n={n} d={d}")
    A = spdgen.covariance(n, d)
    _, sx = spdgen.seeds(5, d)
    Xt = spdgen.rhs(n, 2, sx)
    Bt = spdgen.accurate_product(A, Xt)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(np.ascontiguousarray(Bt)).cuda()
    X, rep, F = spd.posv(Ad, Bd, prec="fp32")
    F.close()
    Xh = X.cpu().numpy()
    Xo, _ = orc.solve(A, Bt)
    _, ro = orc.ir(A, Bt, prec="fp32")
    kappa = cond_bound(n, d)
    fe = float((np.abs(Xh - Xo).max(axis=1) / np.abs(Xo).max(axis=1)).max())
    _say(f"  library {rep.status} {rep.iters_low}/{rep.iters_high}; oracle {ro.status} {ro.iters_low}/{ro.iters_high}; "
         f"|x - x_oracle| {fe:.2e} (bar {10 * kappa * U64:.2e})")
    assert rep.status == 0 and ro.status == 0
    assert rep.prec_used == ro.prec_used == 2 and rep.fallbacks == ro.fallbacks == 0
    assert abs(rep.iters_low - ro.iters_low) <= 1
    assert fe <= 10 * kappa * U64
    assert orc.backward_error(A, Xh, Bt).max() <= 1e-14
