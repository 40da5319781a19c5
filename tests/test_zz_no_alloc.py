"""spd_residual_noalloc (the binary64 residual of Algorithm 1, for
callers that cannot allocate) against spd_residual, through the C ABI: the
same residual bit for bit and the same backward errors, on calls in a row
with shrinking inputs (the static scratch keeps the previous call's
contents), on both residual kernels (1-2 and 3+ right-hand sides), with and
without a caller-provided R."""
import ctypes as C
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _case(n, m, seed):
    import torch
    A = spdgen.logspaced(n, 1e3, seed)
    Xt = spdgen.rhs(n, m, seed + 1)
    Bt = spdgen.accurate_product(A, Xt)
    X = Xt + 1e-7 * spdgen.rhs(n, m, seed + 2)  # an inexact iterate: a nonzero residual
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return dev(A), dev(X), dev(Bt)


def _both(spd, A, X, B, with_R):
    import torch
    lib = spd.load()
    n, m = A.shape[0], X.shape[0]
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = []
    for fn in (lib.spd_residual, lib.spd_residual_noalloc):
        R = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda") if with_R else None
        eta = np.full(m, np.nan)
        s = fn(_ptr(A), n, n, _ptr(X), n, _ptr(B), n, m, _ptr(R) if with_R else None, n,
               eta.ctypes.data_as(C.c_void_p), st)
        torch.cuda.synchronize()
        assert s == 0, (fn, s)
        out.append((None if R is None else R.cpu().numpy(), eta))
    return out


@pytest.mark.parametrize("with_R", [True, False])
def test_noalloc_residual_matches_spd_residual(spd, with_R):
    # larger first, then smaller: the second call must not see the first's data
    for n, m, seed in ((4096, 2, 31), (1500, 1, 41), (2000, 5, 51), (700, 3, 61)):
        _say(f"noalloc residual n={n} m={m} R={'yes' if with_R else 'no'}")
        A, X, B = _case(n, m, seed)
        (R1, e1), (R2, e2) = _both(spd, A, X, B, with_R)
        if with_R:
            assert np.array_equal(R1, R2)
            assert np.all(np.isfinite(R1)) and np.abs(R1).max() > 0
        assert np.array_equal(e1, e2), (e1, e2)
        assert np.all(e1 > 0) and np.all(e1 < 1e-6)


def test_noalloc_residual_rejects_oversize(spd):
    import torch
    lib = spd.load()
    A = torch.zeros(1, dtype=torch.float64, device="cuda")
    # n = 20000 with 2 RHS needs more than the static array: rejected up front
    s = lib.spd_residual_noalloc(_ptr(A), 20000, 20000, _ptr(A), 20000, _ptr(A), 20000, 2, _ptr(A), 20000, None,
                                 None)
    assert s == spd.ERR_INVALID_ARG
