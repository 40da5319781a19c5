"""GPU parity at the benchmark's full size: n = 16384, cond(A) = 1e4, one
right-hand side, binary32 factor with binary64 refinement (Algorithm 1) --
the inputs (same generators and seeds) and the call that bench.py times.

The oracle cannot solve this size in seconds, so it checks outputs it can
compute one by one: the binary64 residual of 64 sampled rows
(oracle.residual_rows on the whole matrix) against the backward-error bar
(eta <= 1e-14), with ||A||_inf from the oracle.  The forward error against
X_true (B = A X_true formed in double-double) is checked over every entry
against 10 cond(A) 2^-53.
"""
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_bench_config_sampled_rows(spd, orc):
    import torch
    n, m, cond = 16384, 1, 1e4
    _say(f"full size posv fp32 n={n} cond={cond:g} m={m}")
    sg, sx = spdgen.seeds(1, 0)
    A = spdgen.logspaced(n, cond, sg, backend="torch", device="cuda")
    Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    X, rep, F = spd.posv(A, B, prec="fp32")
    torch.cuda.synchronize()
    assert rep.status == 0, rep.status
    assert spd.PREC_NAME[rep.prec_used] == "fp32" and rep.fallbacks == 0
    assert rep.eta <= 1e-14
    # forward error, every entry
    fe = float((X - Xt).abs().max() / Xt.abs().max())
    assert fe <= 10 * cond * U64, fe
    # oracle residual of sampled rows
    rng = np.random.Generator(np.random.PCG64(2024))
    rows = np.sort(rng.choice(n, size=64, replace=False))
    rows[0], rows[-1] = 0, n - 1  # both ends of the matrix
    Ah = A.cpu().numpy()
    Xh, Bh = X.cpu().numpy(), B.cpu().numpy()
    R = orc.residual_rows(Ah, Xh, Bh, rows)
    anorm = orc.norminf_sym(Ah)
    eta_rows = float(np.max(np.abs(R)) / (anorm * np.max(np.abs(Xh)) + np.max(np.abs(Bh))))
    _say(f"  iters {rep.iters_low}/{rep.iters_high} eta {rep.eta:.2e} eta(rows, oracle) {eta_rows:.2e} fwd {fe:.2e}")
    assert eta_rows <= 1e-14, eta_rows
