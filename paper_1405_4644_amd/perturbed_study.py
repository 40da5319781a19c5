"""The perturbed-factor experiment of Section 3.1 (Fig. 3(b)) on the library.

For each size n and exponent gamma: factor A in binary64 (spd_factor), take
R = L^T, add a random upper-triangular E scaled so that
||E||_2 / ||R||_2 = 10^gamma, hand R + E back as the factor
(spd_factor_import) and refine with it (spd_refine) until the backward
error reaches binary64 level or Eq. (4) stops holding (divergence), counting
the corrections.  Every step runs in the library's kernels; torch only
allocates device memory and draws E.

    python -m paper_1405_4644_amd.perturbed_study --sizes 1000,4000,16384 \
        --gammas -1,-3.25,-5.5,-7.75,-10 --cond 10

Prints one JSON line per (n, gamma).
"""
import argparse
import json
import math
import time

import paper_1405_4644_amd as spd
import spdgen


def norm2(M, iters=40, seed=0):
    """||M||_2 by power iteration on M^T M (a lower estimate that converges
    to the largest singular value)."""
    import torch
    g = torch.Generator(device=M.device)
    g.manual_seed(seed)
    v = torch.randn(M.shape[1], dtype=M.dtype, device=M.device, generator=g)
    v /= v.norm()
    s = 0.0
    for _ in range(iters):
        w = M.T @ (M @ v)
        s = math.sqrt(float(w.norm()))
        v = w / w.norm()
    return s


def run_case(n, gamma, cond, m, max_iter, seed):
    import torch
    sg, sx = spdgen.seeds(7, seed)
    A = spdgen.logspaced(n, cond, sg, backend="torch", device="cuda")
    Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    F0, info, st = spd.factor(A, prec="fp64", opts=spd.default_opts(equilibrate=0))
    if st != spd.OK:
        return {"n": n, "gamma": gamma, "status": spd.status_str(st), "info": info}
    L, d, mu = spd.export(F0)  # factor of mu D A D
    L = (L / d[:, None]) / math.sqrt(mu)
    del F0
    g = torch.Generator(device="cuda")
    g.manual_seed(1000003 * seed + n)
    E = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g).tril_()
    E *= (10.0 ** gamma) * norm2(L) / norm2(E)
    Lp = (L + E).t().contiguous().t()  # column-major
    del E, L
    F, info, st = spd.factor_import(Lp, prec="fp64")
    if st != spd.OK:
        return {"n": n, "gamma": gamma, "status": spd.status_str(st), "info": info}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X = spd.solve(F, B)
    rep = spd.refine(F, A, B, X, spd.default_opts(max_iter=max_iter, fallback=0))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    fwd = float(((X - Xt).abs().amax(dim=1) / Xt.abs().amax(dim=1)).max())
    return {"n": n, "gamma": gamma, "cond": cond, "m": m, "status": spd.status_str(rep.status),
            "iters_low": rep.iters_low, "iters_high": rep.iters_high, "eta": rep.eta, "fwd": fwd,
            "ms": 1e3 * t}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--sizes", default="1000,4000,16384")
    ap.add_argument("--gammas", default="-1,-3.25,-5.5,-7.75,-10")
    ap.add_argument("--cond", type=float, default=10.0)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    for n in (int(s) for s in a.sizes.split(",")):
        for gamma in (float(s) for s in a.gammas.split(",")):
            print(json.dumps(run_case(n, gamma, a.cond, a.nrhs, a.max_iter, a.seed)), flush=True)


if __name__ == "__main__":
    main()
