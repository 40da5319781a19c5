"""Full-size parity of Algorithm 1 (Section 3.1) in every factor precision
at the sizes the benchmark configurations run:

* n = 16384, log-spaced eigenvalues: binary32 at cond 1e2 / 1e4 / 1e6 with
  1 and 64 right-hand sides (the cond 1e4, 1 RHS case is in
  test_gpu_fullsize.py), binary16 and bfloat16 at cond 1e1 ... 1e4, 1 RHS;
* n = 49152 (19.3 GB in binary64), cond 1e1 / 1e3 / 1e5, binary16 and
  bfloat16 with the fallback chain, 1 RHS.

The oracle cannot factor these sizes in seconds, so each result is checked
by what the oracle computes one row at a time -- the binary64 residual of
64 sampled rows (both ends included) from those rows of A, giving a lower
bound on the backward error -- and by properties that hold at any size: the
forward error against X_true (B = A X_true in double-double) under the bar
10 cond 2^-53, which SPD_OK must imply (the stopping rule), and the
precision the refinement ends in, fixed by Eq. (4) where cond * u_low is
far from one: it must stay in the requested half precision when
cond * u_low <= 0.05 and must fall back to binary32 when cond * u_low >= 10.
"""
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
ULOW = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "fp32": 2.0 ** -24}
_CACHE = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _system(n, cond, m, config):
    """A, X_true, B on the device, generated once per (n, cond, m)."""
    import torch
    key = (n, cond, m, config)
    if key not in _CACHE:
        _CACHE.clear()
        torch.cuda.empty_cache()
        sg, sx = spdgen.seeds(config, 0)
        _say(f"  generating n={n} cond={cond:g} m={m}")
        A = spdgen.logspaced(n, cond, sg, backend="torch", device="cuda")
        Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
        B = spdgen.accurate_product(A, Xt)
        torch.cuda.synchronize()
        _CACHE[key] = (A, Xt, B)
    return _CACHE[key]


def _check(spd, orc, A, Xt, B, X, rep, cond, label):
    import torch
    n = A.shape[0]
    fe = float(((X - Xt).abs().amax(dim=1) / Xt.abs().amax(dim=1)).max())
    rng = np.random.Generator(np.random.PCG64(n + int(cond)))
    rows = np.sort(rng.choice(n, size=64, replace=False))
    rows[0], rows[-1] = 0, n - 1
    ridx = torch.from_numpy(rows).to(A.device)
    Arows = A.index_select(0, ridx).cpu().numpy()  # rows of the symmetric A
    Xh, Bh = X.cpu().numpy(), B.cpu().numpy()
    R = orc.residual_given_rows(Arows, Xh, Bh, rows)
    anorm_lb = float(np.abs(Arows).sum(axis=1).max())  # ||A||_inf >= any row's sum
    den = anorm_lb * np.abs(Xh).max(axis=1) + np.abs(Bh).max(axis=1)
    eta_rows = float((np.abs(R).max(axis=1) / den).max())
    _say(f"  {label}: status {rep.status} prec {spd.PREC_NAME[rep.prec_used]} fallbacks {rep.fallbacks} "
         f"iters {rep.iters_low}/{rep.iters_high} eta {rep.eta:.2e} eta(rows) {eta_rows:.2e} "
         f"fwd {fe:.2e} (bar {10 * cond * U64:.2e})")
    assert rep.status == 0, rep.as_dict()
    assert rep.eta <= 1e-14
    # the rows' residual over a lower bound of ||A|| bounds eta(rows) from above
    assert eta_rows <= 2e-14, eta_rows
    assert fe <= 10 * cond * U64, fe


def _expect_prec(spd, rep, prec, cond):
    used = spd.PREC_NAME[rep.prec_used]
    if cond * ULOW[prec] <= 0.05:
        assert used == prec and rep.fallbacks == 0, rep.as_dict()
    elif cond * ULOW[prec] >= 10:
        assert used == "fp32" and rep.fallbacks == 1, rep.as_dict()
    else:
        assert used in (prec, "fp32"), rep.as_dict()


@pytest.mark.parametrize("cond,m", [(1e2, 1), (1e6, 1), (1e2, 64), (1e4, 64), (1e6, 64)])
def test_config1_fp32_n16384(spd, orc, cond, m):
    n = 16384
    _say(f"config 1: fp32 n={n} cond={cond:g} m={m}")
    A, Xt, B = _system(n, cond, m, 1)
    X, rep, F = spd.posv(A, B, prec="fp32")
    F.close()
    assert spd.PREC_NAME[rep.prec_used] == "fp32" and rep.fallbacks == 0, rep.as_dict()
    _check(spd, orc, A, Xt, B, X, rep, cond, "fp32")


@pytest.mark.parametrize("cond", [1e1, 1e2, 1e3, 1e4])
def test_half_precisions_n16384(spd, orc, cond):
    n = 16384
    _say(f"half precisions n={n} cond={cond:g}")
    A, Xt, B = _system(n, cond, 1, 1)
    for prec in ("fp16", "bf16"):
        X, rep, F = spd.posv(A, B, prec=prec)
        F.close()
        _check(spd, orc, A, Xt, B, X, rep, cond, prec)
        _expect_prec(spd, rep, prec, cond)


@pytest.mark.parametrize("cond", [1e1, 1e3, 1e5])
def test_config2_half_n49152(spd, orc, cond):
    import torch
    n = 49152
    _say(f"config 2: n={n} cond={cond:g}")
    A, Xt, B = _system(n, cond, 1, 2)
    for prec in ("fp16", "bf16"):
        X, rep, F = spd.posv(A, B, prec=prec)
        F.close()
        del F
        torch.cuda.empty_cache()
        _check(spd, orc, A, Xt, B, X, rep, cond, prec)
        _expect_prec(spd, rep, prec, cond)
