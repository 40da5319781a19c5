"""GPU parity of the batched persistent solver (many independent systems,
each through Algorithm 1 in one launch) against the oracle, per system.

Bars (per system, as for the single-system path): eta <= 1e-14 recomputed by
the oracle; forward error <= 10 cond 2^-53 against X_true and the oracle's
binary64 solution; outcome (precision used, fallbacks) equal to the oracle's
emulation of Algorithm 1; iteration counts within 1 (FP32) or at most the
oracle's + 1 (BF16/FP16: the batched factor rounds a subset of the products
the oracle rounds); breakdown column exactly the oracle's; results
independent of the order of the systems in the batch (bitwise); graph replays
bitwise equal to the eager call.
"""
import sys

import numpy as np
import pytest

import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
PREC_ID = {"bf16": 0, "fp16": 1, "fp32": 2, "fp64": 3, "auto": 4}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(pb):
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    return (t(pb.n, torch.int32), t(pb.m, torch.int32), t(pb.a_off, torch.int64), t(pb.A, torch.float64),
            t(pb.b_off, torch.int64), t(pb.B, torch.float64))


def _run(spd, pb, prec, opts=None):
    import torch
    n, m, ao, A, bo, B = _dev(pb)
    if isinstance(prec, (list, tuple)):
        prec = torch.tensor([PREC_ID[p] for p in prec], dtype=torch.int32, device="cuda")
    bt = spd.Batch(n, m, ao, A, bo, B, prec=prec)
    spd.solve_batched(bt, opts)
    torch.cuda.synchronize()
    return bt, bt.X.cpu().numpy(), bt.reports(), bt.prec.cpu().numpy()


def _sys(pb, s):
    n, m = int(pb.n[s]), int(pb.m[s])
    A = pb.A[pb.a_off[s]:pb.a_off[s] + n * n].reshape(n, n)
    B = pb.B[pb.b_off[s]:pb.b_off[s] + n * m].reshape(m, n)
    Xt = pb.Xt[pb.b_off[s]:pb.b_off[s] + n * m].reshape(m, n)
    return A, B, Xt


def _xs(X, pb, s):
    n, m = int(pb.n[s]), int(pb.m[s])
    return X[pb.b_off[s]:pb.b_off[s] + n * m].reshape(m, n)


def _check_system(orc, pb, s, X, rep, prec, exact_iters):
    A, B, Xt = _sys(pb, s)
    cond = float(pb.cond[s])
    Xs = _xs(X, pb, s)
    _, orep = orc.ir(A, B, prec=prec)
    assert rep["status"] == 0 and orep.status == 0, (s, rep, orep)
    assert rep["prec_used"] == orep.prec_used and rep["fallbacks"] == orep.fallbacks, (s, rep, orep)
    if exact_iters:
        assert abs(int(rep["iters_low"]) - orep.iters_low) <= 1, (s, rep, orep)
    else:
        assert int(rep["iters_low"]) <= orep.iters_low + 1, (s, rep, orep)
    eta = orc.backward_error(A, Xs, B)
    assert np.all(eta <= 1e-14), (s, eta)
    bound = 10 * cond * U64
    Xo, info = orc.solve(A, B)
    fe = lambda Y, R: np.max(np.abs(Y - R), axis=1) / np.max(np.abs(R), axis=1)
    assert np.all(fe(Xs, Xo) <= bound), (s, fe(Xs, Xo), bound)
    assert np.all(fe(Xs, Xt) <= bound), (s, fe(Xs, Xt), bound)


EDGE = [(1, 1e1, 1), (2, 1e2, 2), (31, 1e3, 1), (32, 1e4, 3), (33, 1e2, 8), (64, 1e5, 1), (65, 1e6, 2),
        (100, 1e3, 4), (127, 1e4, 1), (128, 1e2, 5), (129, 1e6, 1), (200, 1e4, 7), (257, 1e3, 2), (300, 1e5, 1),
        (512, 1e4, 2), (511, 1e6, 8)]


def test_batched_fp32_matches_oracle(spd, orc):
    shapes = EDGE + spdgen.batch_shapes(24, config=3, nmin=8, nmax=260)
    pb = spdgen.packed_batch(shapes, config=3)
    _say("batched fp32:", len(shapes), "systems")
    bt, X, reps, prec = _run(spd, pb, "fp32")
    assert spd.batched_config(len(shapes)) is not None
    for s in range(len(shapes)):
        _check_system(orc, pb, s, X, reps[s], "fp32", True)
    assert np.all(prec == reps["prec_used"])


def test_batched_half_and_fp64_requests(spd, orc):
    shapes = [(200, 1e1, 1), (150, 1e2, 2), (96, 1e3, 1), (300, 1e3, 3), (64, 1e5, 1), (130, 1e1, 4),
              (257, 1e2, 1), (90, 1e4, 2)]
    precs = ["bf16", "fp16", "fp16", "bf16", "fp16", "fp64", "bf16", "fp64"]
    pb = spdgen.packed_batch(shapes, config=3, first_index=1000)
    bt, X, reps, prec = _run(spd, pb, precs)
    for s, p in enumerate(precs):
        _say(" ", shapes[s], p, dict(zip(reps.dtype.names, reps[s].tolist())))
        _check_system(orc, pb, s, X, reps[s], p, p in ("fp32", "fp64"))
        if p == "fp64":
            assert (int(reps[s]["iters_low"]), int(reps[s]["iters_high"])) == (1, 1)


def test_batched_breakdown_and_limits(spd, orc):
    import torch
    n0 = 120
    Aind = spdgen.indefinite(n0, 77, seed=4)
    shapes = [(50, 1e2, 1), (n0, 1e2, 1), (40, 1e2, 1), (30, 1e2, 2)]
    pb = spdgen.packed_batch(shapes, config=3, first_index=2000)
    pb.A[pb.a_off[1]:pb.a_off[1] + n0 * n0] = Aind.reshape(-1)
    n, m, ao, A, bo, B = _dev(pb)
    # system 2: n beyond the limit; system 3: too many right-hand sides
    n[2] = 513
    m[3] = 9
    bt = spd.Batch(n, m, ao, A, bo, B, prec="fp32")
    spd.solve_batched(bt, spd.default_opts(fallback=0))
    reps = bt.reports()
    assert reps[0]["status"] == 0
    assert reps[1]["status"] == 2 and reps[1]["info"] == 77 and reps[1]["prec_used"] == 2
    assert reps[2]["status"] == 1 and reps[3]["status"] == 1
    # with fallback: FP32 breaks down, then FP64 does
    bt2 = spd.Batch(n, m, ao, A, bo, B, prec="fp32")
    spd.solve_batched(bt2)
    r2 = bt2.reports()
    assert r2[1]["status"] == 2 and r2[1]["info"] == 77 and r2[1]["prec_used"] == 3 and r2[1]["fallbacks"] == 1
    _, orep = orc.ir(Aind, np.ones((1, n0)), prec="fp32", fallback=False)
    assert orep.info == 77


def test_batched_empty_systems(spd):
    import torch
    shapes = [(40, 1e2, 1), (0, 1e2, 1), (30, 1e2, 0), (20, 1e2, 1)]
    pb = spdgen.packed_batch([(40, 1e2, 1), (1, 1e2, 1), (30, 1e2, 1), (20, 1e2, 1)], config=3, first_index=3000)
    n, m, ao, A, bo, B = _dev(pb)
    n[1] = 0
    m[2] = 0
    bt = spd.Batch(n, m, ao, A, bo, B, prec="fp32")
    spd.solve_batched(bt)
    reps = bt.reports()
    assert list(reps["status"]) == [0, 0, 0, 0]
    assert reps[1]["iters_low"] == 0 and reps[2]["iters_low"] == 0


def test_batched_order_invariance(spd):
    shapes = spdgen.batch_shapes(20, config=3, nmin=16, nmax=200)
    pb = spdgen.packed_batch(shapes, config=3, first_index=4000)
    _, X1, r1, _ = _run(spd, pb, "fp32")
    perm = np.random.Generator(np.random.PCG64(5)).permutation(len(shapes))
    pbp = spdgen.packed_batch([shapes[i] for i in perm], config=3, first_index=0)
    # regenerate with the original indices so every system is the same matrix
    for k, i in enumerate(perm):
        n, m = shapes[i][0], shapes[i][2]
        pbp.A[pbp.a_off[k]:pbp.a_off[k] + n * n] = pb.A[pb.a_off[i]:pb.a_off[i] + n * n]
        pbp.B[pbp.b_off[k]:pbp.b_off[k] + n * m] = pb.B[pb.b_off[i]:pb.b_off[i] + n * m]
    _, X2, r2, _ = _run(spd, pbp, "fp32")
    for k, i in enumerate(perm):
        assert np.array_equal(_xs(X2, pbp, k), _xs(X1, pb, i)), (k, i)
        assert r2[k]["iters_low"] == r1[i]["iters_low"]


def test_batched_only_lower_triangle_read(spd):
    # every system's strict upper triangle (element (i, j), i < j, at
    # A[i + j n]) poisoned with NaN: the solutions must be bit for bit those
    # of the symmetric matrices, in every precision and with the picker
    shapes = spdgen.batch_shapes(24, config=3, nmin=16, nmax=300)
    pb = spdgen.packed_batch(shapes, config=3, first_index=4500)
    poisoned = pb.A.copy()
    for s, (n, _, _) in enumerate(shapes):
        blk = poisoned[pb.a_off[s]:pb.a_off[s] + n * n].reshape(n, n)  # blk[j, i] = element (i, j)
        blk[np.tril_indices(n, -1)] = np.nan  # rows j > i of blk: elements with i < j
    for prec in ("fp32", "fp64", "fp16"):
        _, X1, r1, _ = _run(spd, pb, prec)
        pbn = spdgen.PackedBatch(pb.n, pb.m, pb.cond, pb.a_off, pb.b_off, poisoned, pb.B, pb.Xt)
        _, X2, r2, _ = _run(spd, pbn, prec)
        assert np.all(r2["status"] == 0), prec
        assert np.array_equal(X1, X2), prec
    spd.picker_load()
    try:
        _, X1, _, p1 = _run(spd, pb, "auto")
        _, X2, _, p2 = _run(spd, spdgen.PackedBatch(pb.n, pb.m, pb.cond, pb.a_off, pb.b_off, poisoned, pb.B, pb.Xt),
                            "auto")
    finally:
        spd.picker_set(None)
    assert np.array_equal(p1, p2) and np.array_equal(X1, X2)


def test_batched_graph_replay(spd):
    import torch
    shapes = spdgen.batch_shapes(16, config=3, nmin=16, nmax=160)
    pb = spdgen.packed_batch(shapes, config=3, first_index=5000)
    n, m, ao, A, bo, B = _dev(pb)
    bt = spd.Batch(n, m, ao, A, bo, B, prec="fp32")
    spd.solve_batched(bt)  # warm: workspace and launch shape
    torch.cuda.synchronize()
    Xe = bt.X.clone()
    re = bt.reps.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.prec.fill_(PREC_ID["fp32"])
            spd.solve_batched(bt)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        bt.X.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bt.X, Xe), rep
        assert torch.equal(bt.reps, re), rep
        _ = (bt.X * 2).sum().item()  # eager work between replays
