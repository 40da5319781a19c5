"""Error paths of the library on the GPU, forced from the host so that every
kernel still ends normally:

* a triangular-solve wait that gives up (the bounded waits of the blocked
  substitutions, limit set to zero) is reported as SPD_ERR_DEVICE by the
  refinement, and a new factorisation of the handle clears it;
* batched calls on two streams share the device's workspace and are ordered
  by the library: both give the oracle's outcome.
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


def test_wait_timeout_reported_and_cleared(spd):
    import torch
    n, cond = 8192, 1e2
    _say(f"wait limit 0: n={n}")
    sg, sx = spdgen.seeds(1, 7)
    A = spdgen.logspaced(n, cond, sg, backend="torch", device="cuda")
    Xt = spdgen.rhs(n, 1, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    F, info, st = spd.factor(A, prec="fp32")
    assert info == 0
    F.set_wait_limit(0.0)  # every wait that is not already satisfied gives up
    X = spd.solve(F, B)
    rep = spd.refine(F, A, B, X, spd.default_opts(fallback=0))
    torch.cuda.synchronize()
    _say(f"  status {rep.status}")
    assert rep.status == spd.ERR_DEVICE
    # a new factor clears the flag; with the default limit the solve is right
    F.set_wait_limit(1.0)
    F, info, st = spd.factor(A, prec="fp32", F=F)
    X = spd.solve(F, B)
    rep = spd.refine(F, A, B, X)
    torch.cuda.synchronize()
    fe = float((X - Xt).abs().max() / Xt.abs().max())
    _say(f"  after re-factor: status {rep.status} iters {rep.iters_low}/{rep.iters_high} fwd {fe:.2e}")
    assert rep.status == 0 and fe <= 10 * cond * U64
    F.close()


def test_batched_calls_on_two_streams(spd, orc):
    import torch
    shapes = spdgen.batch_shapes(96, config=3, nmin=32, nmax=256)
    pb = spdgen.packed_batch(shapes, config=3, first_index=7000)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    n, m, ao, A, bo = (t(pb.n, torch.int32), t(pb.m, torch.int32), t(pb.a_off, torch.int64),
                       t(pb.A, torch.float64), t(pb.b_off, torch.int64))
    B1 = t(pb.B, torch.float64)
    B2 = 2.0 * B1  # solution 2 X_true
    bt1 = spd.Batch(n, m, ao, A, bo, B1, prec="fp32")
    spd.solve_batched(bt1)  # first call: autotune, workspace
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    bt1 = spd.Batch(n, m, ao, A, bo, B1, prec="fp32")
    bt2 = spd.Batch(n, m, ao, A, bo, B2, prec="fp32")
    with torch.cuda.stream(s1):
        spd.solve_batched(bt1)
    with torch.cuda.stream(s2):
        spd.solve_batched(bt2)
    torch.cuda.synchronize()
    X1, X2 = bt1.X.cpu().numpy(), bt2.X.cpu().numpy()
    r1, r2 = bt1.reports(), bt2.reports()
    for s in range(len(shapes)):
        k, nn = int(pb.b_off[s]), int(pb.n[s]) * int(pb.m[s])
        Xt = pb.Xt[k:k + nn]
        bar = 10 * float(pb.cond[s]) * U64
        assert r1[s]["status"] == 0 and r2[s]["status"] == 0, (s, r1[s], r2[s])
        scale = np.abs(Xt).max()
        assert np.abs(X1[k:k + nn] - Xt).max() / scale <= bar, s
        assert np.abs(X2[k:k + nn] - 2.0 * Xt).max() / (2.0 * scale) <= bar, s
