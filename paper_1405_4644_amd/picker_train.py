"""Train the precision picker of the batched solver (SPD_AUTO) on data the
method generates itself.

    python -m paper_1405_4644_amd.picker_train [--systems 200000] [--out DIR]

1. Draw systems from the batched workload's distribution (n ~ U{32..512},
   cond ~ 10^U(1, 6) with log-spaced spectra, 1..8 right-hand sides) in
   chunks of 4096 (seeds disjoint from the evaluation batch).
2. Label each system by running the batched solver at every precision
   (BF16, FP16, FP32, FP64; no fallback) and timing each system on the
   device (the least of --repeats runs): the label is the cheapest
   precision that reached the binary64 backward error within 10
   corrections; among precisions within 2 % of the cheapest, the highest.
3. Train the perceptron with the library's own kernels (spd_mlp_grad,
   spd_mlp_adam; mini-batches, Adam).
4. Evaluate on the held-out batch (the workload's own 4096 systems): share of
   mispicks, and the measured cost of picking against always FP32 and
   always FP64 (a failed pick costs its own run plus the FP64 fallback).

Writes DIR/picker_weights.npz (params, feature normalisation is part of the
features) and DIR/picker_report.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PRECS = ("bf16", "fp16", "fp32", "fp64")
WEIGHTS = os.path.join(HERE, "picker_weights.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def label_rule(conv, cost):
    """Cheapest converged precision; ties within 2 % go to the higher one."""
    y = np.full(len(conv), 3, dtype=np.int32)
    for s in range(len(conv)):
        cand = [k for k in range(4) if conv[s, k]]
        if cand:
            best = min(cost[s, k] for k in cand)
            y[s] = max(k for k in cand if cost[s, k] <= 1.02 * best)
    return y


def outcomes(spd, pb, repeats=3):
    """Features, convergence and per-system ticks at every precision; each
    system's ticks are the least over `repeats` runs (workgroups sharing a
    compute unit perturb a single run's clocks)."""
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    n, m, ao, bo = t(pb.n, torch.int32), t(pb.m, torch.int32), t(pb.a_off, torch.int64), t(pb.b_off, torch.int64)
    A = pb.A if isinstance(pb.A, torch.Tensor) else t(pb.A, torch.float64)
    B = pb.B if isinstance(pb.B, torch.Tensor) else t(pb.B, torch.float64)
    bt = spd.Batch(n, m, ao, A, bo, B, prec="fp32")
    feat = spd.picker_features(bt).cpu().numpy()
    conv = np.zeros((bt.batch, 4), dtype=bool)
    ticks = np.full((bt.batch, 4), np.iinfo(np.int64).max, dtype=np.int64)
    tk = torch.zeros(bt.batch, dtype=torch.int64, device="cuda")
    opts = spd.default_opts(fallback=0)
    for k, p in enumerate(PRECS):
        conv[:, k] = True
        for _ in range(repeats):
            bt.prec.fill_(spd.PREC[p])
            spd.solve_batched(bt, opts, ticks=tk)
            conv[:, k] &= bt.reports()["status"] == 0
            ticks[:, k] = np.minimum(ticks[:, k], tk.cpu().numpy())
    return feat, conv, ticks, bt


def train(spd, X, y, epochs=40, batch=2048, lr=3e-3, seed=0):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    # He-style initialisation of the three layers, zero biases
    p = np.zeros(spd.PICKER_NPARAM, dtype=np.float32)
    o = 0
    for fan_in, fan_out in ((16, 64), (64, 64), (64, 4)):
        p[o:o + fan_in * fan_out] = rng.normal(0, np.sqrt(2.0 / fan_in), fan_in * fan_out)
        o += fan_in * fan_out + fan_out
    P = torch.from_numpy(p).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    yd = torch.from_numpy(y.astype(np.int32)).cuda()
    N = len(y)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch]
            g, loss = spd.mlp_grad(P, Xd[idx].contiguous(), yd[idx].contiguous())
            step += 1
            spd.mlp_adam(P, g, M, V, step, lr=lr)
        acc = float((spd.mlp_forward(P, Xd).argmax(dim=1) == yd.long()).float().mean())
        hist.append((ep, float(loss.item()), acc))
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"epoch {ep}: loss {float(loss.item()):.4f} train accuracy {acc:.4f}")
    return P, hist


def costs(pick, conv, ticks):
    """Per-system cost of running `pick` (a failed pick adds the FP64 run)."""
    c = ticks[np.arange(len(pick)), pick].astype(np.float64)
    fail = ~conv[np.arange(len(pick)), pick]
    c[fail] += ticks[fail, 3]
    return c


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--systems", type=int, default=200000)
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--repeats", type=int, default=3, help="timed runs per precision; each system keeps the least")
    ap.add_argument("--out", default=HERE)
    args = ap.parse_args()
    import torch

    import paper_1405_4644_amd as spd
    import spdgen
    spd.load()
    torch.cuda.set_device(0)
    t0 = time.time()
    feats, convs, tickss = [], [], []
    nchunk = (args.systems + args.chunk - 1) // args.chunk
    for c in range(nchunk):
        k = min(args.chunk, args.systems - c * args.chunk)
        shapes = spdgen.batch_shapes(k, config=100 + c)
        pb = spdgen.packed_batch_grouped(shapes, seed=100 + c)
        f, cv, tk, _ = outcomes(spd, pb, args.repeats)
        feats.append(f)
        convs.append(cv)
        tickss.append(tk)
        del pb
        torch.cuda.empty_cache()
        log(f"chunk {c + 1}/{nchunk}: {k} systems labelled ({time.time() - t0:.0f} s)")
    X = np.concatenate(feats)
    conv = np.concatenate(convs)
    ticks = np.concatenate(tickss)
    y = label_rule(conv, ticks)
    log("label histogram (bf16, fp16, fp32, fp64):", np.bincount(y, minlength=4).tolist())
    P, hist = train(spd, X, y, epochs=args.epochs)
    params = P.cpu().numpy()
    # held-out: the batched workload's own systems (exact per-system recipe)
    shapes = spdgen.batch_shapes(4096, config=3)
    pb = spdgen.packed_batch(shapes, config=3, backend="torch", device="cuda")
    fh, ch, th, bt = outcomes(spd, pb, args.repeats)
    yh = label_rule(ch, th)
    pick = spd.mlp_forward(P, torch.from_numpy(fh).cuda()).argmax(dim=1).cpu().numpy()
    cost_pick = costs(pick, ch, th).sum()
    cost_fp32 = costs(np.full(len(pick), 2), ch, th).sum()
    cost_fp64 = costs(np.full(len(pick), 3), ch, th).sum()
    cost_best = costs(yh, ch, th).sum()
    # wall clock of whole batched calls (with the fallback chain)
    def wall(prec, picker_on):
        spd.picker_set(P if picker_on else None)
        ts = []
        for _ in range(3):
            bt.prec.fill_(spd.PREC[prec])
            torch.cuda.synchronize()
            t = time.perf_counter()
            spd.solve_batched(bt)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        ok = bool((bt.reports()["status"] == 0).all())
        spd.picker_set(None)
        return float(np.median(ts)), ok
    w_auto, ok_auto = wall("auto", True)
    w_fp32, ok_fp32 = wall("fp32", False)
    w_fp64, ok_fp64 = wall("fp64", False)
    report = {
        "training_systems": int(len(y)), "label_repeats": args.repeats,
        "label_histogram": np.bincount(y, minlength=4).tolist(),
        "final_train_loss": hist[-1][1], "final_train_accuracy": hist[-1][2],
        "heldout_systems": int(len(yh)), "heldout_label_histogram": np.bincount(yh, minlength=4).tolist(),
        "heldout_pick_histogram": np.bincount(pick, minlength=4).tolist(),
        "heldout_mispick_rate": float(np.mean(pick != yh)),
        "heldout_pick_fails": int((~ch[np.arange(len(pick)), pick]).sum()),
        "heldout_cost_ratio_vs_fp32": float(cost_pick / cost_fp32),
        "heldout_cost_ratio_vs_fp64": float(cost_pick / cost_fp64),
        "heldout_cost_ratio_best_vs_fp32": float(cost_best / cost_fp32),
        "heldout_wall_ms": {"auto": w_auto * 1e3, "fp32": w_fp32 * 1e3, "fp64": w_fp64 * 1e3},
        "heldout_all_converged": {"auto": ok_auto, "fp32": ok_fp32, "fp64": ok_fp64},
        "seconds": time.time() - t0,
    }
    os.makedirs(args.out, exist_ok=True)
    np.savez(os.path.join(args.out, "picker_weights.npz"), params=params,
             label_histogram=np.bincount(y, minlength=4))
    with open(os.path.join(args.out, "picker_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
