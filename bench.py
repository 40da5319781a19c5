#!/usr/bin/env python3
"""Benchmark: time to a binary64-accurate solve and effective TFLOP/s of
mixed-precision Cholesky with iterative refinement (Algorithm 1 of the paper)
against plain binary64 Cholesky on the same GPU, dense SPD n = 16384.

One step = one whole solve of A X = B with A, B already resident in HBM:
equilibrate/convert, low-precision factorisation, first solve, and the
binary64 refinement loop until the backward error reaches binary64 level.

    python bench.py [--steps K] [--warmup W] [--n 16384] [--cond 1e4] [--nrhs 1]
    python bench.py --workload covariance [--decay 1|2|4]   # Section 4 matrix, n=70000, 32 RHS
    python bench.py --workload covariance --solver cg [--band 16] [--nrhs 1]
                                     # Algorithm 2 (CG-IR), dense or banded binary32 operator

Prints ONE JSON line on stdout (progress goes to stderr).  `value` is the
effective rate F(n, m) / t_step with F = n^3/3 + n^2/2 + n/6 + 2 n^2 m (the
binary64 algorithm's flops, LINPACK style).  `roofline` describes the
dominant kernel (the MFMA trailing update), timed with HIP events around its
launches inside the timed region.  `cpu_baseline` is the CPU oracle (plain
binary64 Cholesky + substitution) timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "fp16": 2500.0, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algo_flops(n: int, m: int) -> float:
    return n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0 + 2.0 * n ** 2 * m


def cpu_baseline_leg(args, A_dev, X_dev, B_dev, rows_check=True):
    """The only part of the benchmark that runs the CPU oracle: (1) the oracle's
    binary64 solve timed on a bounded sample system of the same recipe, and
    (2) the oracle's residual on sampled rows of the GPU solution (it reads
    the whole matrix on the host: skipped above n = 32768)."""
    import numpy as np

    import oracle
    oracle.lib()
    # sample: the leading ns x ns principal block of the benchmark matrix (SPD,
    # same spectrum shape), right-hand sides = that block times X_true's head
    ns = min(args.cpu_sample_n, A_dev.shape[0])
    As = np.ascontiguousarray(A_dev[:ns, :ns].cpu().numpy())
    Xs = np.random.Generator(np.random.PCG64(11)).standard_normal((args.nrhs, ns))
    Bs = Xs @ As
    t0 = time.perf_counter()
    X, info = oracle.solve(As, Bs)
    t = time.perf_counter() - t0
    rate = algo_flops(ns, args.nrhs) / t / 1e12
    cores = oracle.threads()
    log(f"cpu oracle: n={ns} solve {t:.2f} s -> {rate * 1e3:.3f} GFLOP/s on {cores} threads")
    cpu = {"value": rate, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"oracle binary64 Cholesky + substitution (potrf+potrs) of the leading {ns} x {ns} "
                     f"principal block of the benchmark matrix, {args.nrhs} RHS, {t:.1f} s; "
                     f"rate = F(n,m)/t at that n"}
    # the same oracle on one core, on a smaller leading block (about 5 s)
    n1 = min(args.cpu_sample_n_1core, ns)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.solve(np.ascontiguousarray(As[:n1, :n1]), Bs[:, :n1])
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    rate1 = algo_flops(n1, args.nrhs) / t1 / 1e12
    log(f"cpu oracle, 1 core: n={n1} solve {t1:.2f} s -> {rate1 * 1e3:.3f} GFLOP/s")
    cpu["one_core"] = {"value": rate1, "unit": "TFLOP/s", "cores": 1,
                       "sample": f"the leading {n1} x {n1} block, {t1:.1f} s"}
    if not rows_check:
        return cpu, None
    # oracle check of the GPU result on sampled rows
    n = A_dev.shape[0]
    rng = np.random.Generator(np.random.PCG64(7))
    rows = np.sort(rng.choice(n, size=min(64, n), replace=False))
    A = A_dev.cpu().numpy()
    Xh = X_dev.cpu().numpy()
    Bh = B_dev.cpu().numpy()
    R = oracle.residual_rows(A, Xh, Bh, rows)
    anorm_rows = np.abs(A[rows, :]).sum(axis=1).max()
    eta_rows = float(np.max(np.abs(R)) / (anorm_rows * np.max(np.abs(Xh)) + np.max(np.abs(Bh))))
    return cpu, {"rows": int(rows.size), "max_abs_residual": float(np.max(np.abs(R))),
                 "eta_lower_bound_rows": eta_rows}


def cg_leg(args, spd, spdgen, torch, A, Xt, B):
    """Algorithm 2 (CG with iterative refinement) on the same system: one step
    = build the binary32 operator (dense, or the band |i - j| <= band) and
    refine X from zero to eta <= 1e-14.  The roofline is the product kernel
    (HBM-bound: A~ is read once per product), timed with HIP events around its
    launches in a second pass of the same steps."""
    n, m = A.shape[0], B.shape[0]
    H = spd.CG()
    X = torch.zeros_like(B)

    def step():
        X.zero_()
        spd.cg_prepare(A, half_band=args.band, H=H)
        return spd.cg_refine(H, A, B, X)[1]

    for _ in range(args.warmup):
        rep = step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        rep = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    spd.profile_reset()
    spd.profile_enable(True)
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt_prof = (time.perf_counter() - t) / args.steps
    spd.profile_enable(False)
    launches, ms, fl, by = spd.profile_query(spd.K_CG_MV)
    H.close()
    fwd = float(((X - Xt).abs().amax(dim=1) / Xt.abs().amax(dim=1)).max())
    log(f"cg band={args.band}: {dt * 1e3:.2f} ms/solve, iters {rep.iters_low}/{rep.iters_high}, eta {rep.eta:.2e}, "
        f"status {rep.status}, product {launches} launches {ms / max(launches, 1) * 1e3:.1f} us each")
    gbs = by / ms / 1e6 if ms > 0 else 0.0
    kind = "dense" if args.band < 0 or args.band >= n - 1 else f"band |i-j| <= {args.band}"
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.lib()
        ns, ms_ = min(args.cpu_sample_n, n), min(m, 4)
        As = spdgen.covariance(ns, args.decay) if args.workload == "covariance" else \
            np.ascontiguousarray(A[:ns, :ns].cpu().numpy())
        Xs = spdgen.rhs(ns, ms_, 17)
        Bs = spdgen.accurate_product(As, Xs)
        t = time.perf_counter()
        _, orep = oracle.cg_ir(As, Bs, half_band=args.band)
        tc = time.perf_counter() - t
        w = (n / ns) * (n if kind == "dense" else 2 * args.band + 1) / (ns if kind == "dense" else 2 * args.band + 1)
        cpu = {"value": tc * 1e3 * w * (m / ms_), "unit": "ms per solve (scaled)", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"oracle.cg_ir on the n={ns} {args.workload} matrix with {ms_} RHS ({kind} operator): "
                         f"{tc:.2f} s, {orep.iters_low}/{orep.iters_high} iterations; scaled by the product's "
                         f"work ratio {w:.0f} and the RHS ratio {m / ms_:g}"}
    return {
        "metric": f"time to FP64-accurate solve, CG with iterative refinement (Algorithm 2, {kind} binary32 "
                  f"operator), n={n}, m={m}",
        "value": dt * 1e3, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload} matrix, d={args.decay}, n={n}, {m} RHS, CG-IR with {kind} "
                               f"binary32 operator, binary64 vectors and residuals",
                   "n": n, "nrhs": m, "band": args.band, "decay": args.decay},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("k_cg_mv_valu" if m <= 4 else "k_cg_mv_mfma_ks + k_cg_mv_ksum") if kind == "dense" else "k_cg_mv_band",
                     "launches": launches, "avg_launch_ms": ms / max(launches, 1),
                     "timed_with_events_ms_per_step": dt_prof * 1e3,
                     "algorithmic_bytes_per_launch": by / max(launches, 1),
                     "tflops": fl / ms / 1e9 if ms > 0 else 0.0},
        "cpu_baseline": cpu,
        "accuracy": {"status": rep.status, "iters": [rep.iters_low, rep.iters_high], "eta": rep.eta,
                     "fwd_err_vs_xtrue": fwd},
    }


def use_shipped_tune_cache():
    """Unless SPD_TUNE_CACHE is set, point it at a private copy of the
    schedule cache shipped with the package (written on an MI355X by
    `python -m paper_1405_4644_amd.tune_cache`), so that the timed runs and
    the committed counter runs use the same schedule.  Returns the source."""
    import shutil
    import tempfile
    if os.environ.get("SPD_TUNE_CACHE"):
        return "SPD_TUNE_CACHE"
    shipped = os.path.join(ROOT, "paper_1405_4644_amd", "tune_cache.json")
    if not os.path.exists(shipped):
        return None
    fd, tmp = tempfile.mkstemp(prefix="spd_tune_", suffix=".json")
    os.close(fd)
    shutil.copyfile(shipped, tmp)
    os.environ["SPD_TUNE_CACHE"] = tmp
    return "paper_1405_4644_amd/tune_cache.json"


def measured_traffic(prec, schedule=None):
    """HBM bytes per launch of the update kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None when
    there is none for this precision, the kernel source changed since, or the
    factorisation ran under another schedule (panels per group, workgroup cap)
    than the counters did."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_k_syrk_update_{prec}_n16384.json")  # written from rocprofv3 --pmc runs
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_1405_4644_amd", "csrc", "k_update.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    if schedule is not None and rec.get("schedule") != schedule:
        return None
    return rec.get("traffic_bytes_per_launch"), rec.get("input")


def kernel_summary(spd, prec):
    """Live per-class kernel figures from the library's HIP events (stream of
    each launch) over the evented steps: launches, average duration, and the
    fraction of the MFMA peak (contractions) or of HBM (the rest) that their
    algorithmic flops / bytes reach."""
    peak = PEAK_TFLOPS[prec]
    out = {}
    for name, k, bound in (("trailing_update", spd.K_UPDATE, "mfma"), ("chain_update", spd.K_CHAIN_UPDATE, "mfma"),
                           ("residual", spd.K_RESIDUAL, "hbm"), ("triangular_solves", spd.K_TRSV, "hbm"),
                           ("convert", spd.K_CONVERT, "hbm")):
        launches, ms, fl, by = spd.profile_query(k)
        if not launches or ms <= 0:
            continue
        d = {"launches": launches, "avg_ms": ms / launches, "total_ms": ms}
        if bound == "mfma":
            d.update(bound="mfma", tflops=fl / ms / 1e9, peak_tflops=peak, frac=fl / ms / 1e9 / peak)
        else:
            d.update(bound="hbm", gbs=by / ms / 1e6, peak_gbs=HBM_PEAK_GBS, frac=by / ms / 1e6 / HBM_PEAK_GBS)
        out[name] = d
    return out


def external_fp64_leg(args, torch, A, B, Xt):
    """A library binary64 Cholesky for context (torch.linalg.cholesky +
    cholesky_solve, i.e. the ROCm solver library): not this project's code."""
    ts = []
    X = None
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        L = torch.linalg.cholesky(A)
        X = torch.cholesky_solve(B.T, L).T
        torch.cuda.synchronize()
        if i >= args.warmup:
            ts.append(time.perf_counter() - t)
        del L
    dt = float(np.median(ts))
    fwd = float((X - Xt).abs().max() / Xt.abs().max())
    log(f"external fp64 (torch.linalg.cholesky + cholesky_solve): {dt * 1e3:.2f} ms/solve")
    return {"ms_per_step": dt * 1e3, "value": algo_flops(A.shape[0], B.shape[0]) / dt / 1e12,
            "fwd_err": fwd, "kind": "library binary64 Cholesky (torch.linalg.cholesky + torch.cholesky_solve "
                                    "on ROCm), context only"}


def energy_leg(args, spd, torch, systems, window):
    """Energy to solution per solve from the GPU's energy accumulator (the
    power-trace method: each configuration repeated for `window` seconds,
    steady-state power from the accumulator's publications), with the idle
    draw measured the same way.  systems: [(label, prec, A, B, flops)]."""
    from paper_1405_4644_amd.power_trace import PowerMonitor
    mon = PowerMonitor(0.002)
    mon.start()
    try:
        mon.phase("idle", lambda: time.sleep(0.05), window)
        for label, prec, A, B, fl in systems:
            F = spd.Factor()
            X = torch.empty_like(B)
            spd.posv(A, B, prec=prec, F=F, X=X)
            mon.phase(label, lambda: spd.posv(A, B, prec=prec, F=F, X=X), window)
            F.close()
    finally:
        mon.stop()
    rep = {p["phase"]: p for p in mon.report()}
    idle = rep["idle"]["avg_watts"]
    out = {"idle_watts": idle, "window_s": window, "method": "GPU socket energy accumulator (amdsmi), "
           "steady state over repeated solves; GPU board only, host not included"}
    for label, prec, A, B, fl in systems:
        p = rep[label]
        j = p["joules"]
        out[label] = {"prec": prec, "ms_per_solve": p["seconds"] * 1e3, "avg_watts": p["avg_watts"],
                      "joules_per_solve": j,
                      "joules_above_idle": (j - idle * p["seconds"]) if (j is not None and idle) else None,
                      "tflops_per_watt": (fl / p["seconds"] / 1e12 / p["avg_watts"]) if p["avg_watts"] else None}
        log(f"energy {label}: {p['avg_watts']:.0f} W, {j:.2f} J/solve" if j else f"energy {label}: n/a")
    return out


def batched_leg(args, spd, spdgen, torch):
    """The many-small-systems workload: 4096 SPD systems, n ~ U{32..512},
    cond ~ 10^U(1, 6), 1..8 right-hand sides, each through Algorithm 1 in one
    persistent launch: FP32 (+ FP64 refinement), FP64 in the same kernel, the
    shipped picker (AUTO), and a host loop of single-system FP64 solves."""
    t0 = time.perf_counter()
    shapes = spdgen.batch_shapes(args.batch, config=3)
    pb = spdgen.packed_batch(shapes, config=3, backend="torch", device="cuda")
    tt = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    bt = spd.Batch(tt(pb.n, torch.int32), tt(pb.m, torch.int32), tt(pb.a_off, torch.int64), pb.A,
                   tt(pb.b_off, torch.int64), pb.B, prec="fp32")
    torch.cuda.synchronize()
    log(f"batched: generated {args.batch} systems in {time.perf_counter() - t0:.1f} s")
    flops = float(sum(algo_flops(n, m) for n, _, m in shapes))

    def timed(prec, picker=False, reps=5):
        if picker:
            spd.picker_load()
        try:
            bt.prec.fill_(spd.PREC[prec])
            spd.solve_batched(bt)  # warm (first call: workspace + launch shape)
            ts = []
            for _ in range(reps):
                bt.prec.fill_(spd.PREC[prec])
                torch.cuda.synchronize()
                t = time.perf_counter()
                spd.solve_batched(bt)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
        finally:
            if picker:
                spd.picker_set(None)
        r = bt.reports()
        return {"ms": float(np.median(ts)) * 1e3, "all_ok": bool((r["status"] == 0).all()),
                "iters_low_mean": float(r["iters_low"].mean()),
                "prec_used": np.bincount(r["prec_used"], minlength=4).tolist(),
                "eff_TFLOPs": flops / float(np.median(ts)) / 1e12}

    out = {"workload": f"{args.batch} SPD systems, n ~ U{{32..512}}, cond ~ 10^U(1,6), 1..8 RHS",
           "fp32": timed("fp32"), "fp64_same_kernel": timed("fp64")}
    import os as _os
    if _os.path.exists(spd.PICKER_WEIGHTS):
        out["auto_picker"] = timed("auto", picker=True)
    out["launch_shape"] = spd.batched_config(args.batch)
    # host loop of single-system FP64 solves over a bounded sample, scaled
    k = min(args.batch, args.loop_sample)
    F = spd.Factor()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s in range(k):
        n, m = int(pb.n[s]), int(pb.m[s])
        A = pb.A[pb.a_off[s]:pb.a_off[s] + n * n].view(n, n)
        B = pb.B[pb.b_off[s]:pb.b_off[s] + n * m].view(m, n)
        spd.posv(A, B, prec="fp64", F=F)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    F.close()
    out["fp64_host_loop"] = {"ms": dt * 1e3 * args.batch / k, "sample_systems": k,
                             "note": "spd_posv(FP64) per system in a host loop, time scaled to the batch"}
    out["speedup_fp32_vs_loop"] = out["fp64_host_loop"]["ms"] / out["fp32"]["ms"]
    log(f"batched: fp32 {out['fp32']['ms']:.2f} ms, fp64 {out['fp64_same_kernel']['ms']:.2f} ms, "
        f"loop {out['fp64_host_loop']['ms']:.1f} ms")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="16384 (70000 for --workload covariance)")
    ap.add_argument("--cond", type=float, default=1e4)
    ap.add_argument("--nrhs", type=int, default=None, help="1 (32 for --workload covariance)")
    ap.add_argument("--workload", choices=["logspaced", "covariance"], default="logspaced",
                    help="logspaced: the headline matrix; covariance: the paper's Section 4 model "
                         "covariance matrix 1/|i-j|^d, 1+sqrt(i) on the diagonal")
    ap.add_argument("--decay", type=int, choices=[1, 2, 4], default=1, help="d of --workload covariance")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--solver", choices=["cholesky", "cg"], default="cholesky",
                    help="cholesky: Algorithm 1 (the default); cg: Algorithm 2 on the same system")
    ap.add_argument("--band", type=int, default=-1, help="--solver cg: half-bandwidth of the operator (-1 dense)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the binary64 baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=8192)
    ap.add_argument("--cpu-sample-n-1core", type=int, default=3072)
    ap.add_argument("--no-half", action="store_true", help="skip the binary16 leg (cond 1e2 system)")
    ap.add_argument("--half-cond", type=float, default=1e2)
    ap.add_argument("--no-energy", action="store_true", help="skip energy per solve")
    ap.add_argument("--energy-window", type=float, default=2.5)
    ap.add_argument("--no-external", action="store_true", help="skip the library binary64 Cholesky")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default schedule)")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-small-systems leg")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--loop-sample", type=int, default=512)
    ap.add_argument("--input", choices=["logspaced", "dominant"], default="logspaced",
                    help="logspaced: Q diag(lambda) Q^T (the workload); dominant: (R + R^T)/2 + n I with R ~ U(-1, 1), "
                         "same sizes, no QR (for hardware-counter runs, whose traffic does not depend on the values)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 3 times (calibrates HBM counters) and exit")
    args = ap.parse_args()
    tune_source = use_shipped_tune_cache()
    cov = args.workload == "covariance"
    if args.n is None:
        args.n = 70000 if cov else 16384
    if args.nrhs is None:
        args.nrhs = 32 if cov else 1

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this solver runs on one GPU (requested --gpus {args.gpus}, WORLD_SIZE {world}); "
              "runs over several GPUs are not supported.", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": args.calibrate_copy, "copies": 3}), flush=True)
        return

    import paper_1405_4644_amd as spd
    import spdgen

    spd.load()
    torch.cuda.set_device(0)
    n, m, cond = args.n, args.nrhs, args.cond
    t0 = time.perf_counter()
    sg, sx = spdgen.seeds(1, 0)
    if cov:
        A = spdgen.covariance(n, args.decay, backend="torch", device="cuda")
        _, sx = spdgen.seeds(5, args.decay)
        cond = spdgen.covariance_cond_bound(n, args.decay)  # a bound: the forward-error bar uses it
    elif args.input == "dominant":
        gen = torch.Generator(device="cuda")
        gen.manual_seed(sg)
        A = torch.rand(n, n, dtype=torch.float64, device="cuda", generator=gen) * 2.0 - 1.0
        A = 0.5 * (A + A.T) + n * torch.eye(n, dtype=torch.float64, device="cuda")
    else:
        A = spdgen.logspaced(n, cond, sg, backend="torch", device="cuda")
    Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    torch.cuda.synchronize()
    log(f"generated {args.workload} n={n} cond{'<=' if cov else '='}{cond:g} m={m} "
        f"in {time.perf_counter() - t0:.1f} s")

    if args.solver == "cg":
        print(json.dumps(cg_leg(args, spd, spdgen, torch, A, Xt, B)), flush=True)
        return

    def run(prec, steps, warmup, profile):
        F = spd.Factor()
        X = torch.empty_like(B)
        rep = None
        for _ in range(warmup):
            X, rep, F = spd.posv(A, B, prec=prec, F=F, X=X)
        torch.cuda.synchronize()
        if profile:
            spd.profile_reset()
            spd.profile_enable(True)
        t = time.perf_counter()
        for _ in range(steps):
            X, rep, F = spd.posv(A, B, prec=prec, F=F, X=X)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        if profile:
            spd.profile_enable(False)
        F.close()
        return dt, rep, X

    # the autotuner's schedule for this order (binary32 and, for its leg,
    # binary16), chosen before any timed step
    tuned = {}
    if not args.no_tune:
        for p in ([args.prec] + (["fp16"] if (args.prec == "fp32" and not args.no_half and not cov) else []) +
                  ([] if args.no_fp64 else ["fp64"])):
            t = time.perf_counter()
            tuned[p] = spd.autotune(n, p)
            tuned[p]["tuning_s"] = time.perf_counter() - t
            log(f"autotune {p}: {tuned[p]}")

    # the headline steps run without per-kernel events; the same number of
    # steps then runs again with events around every trailing-update and
    # residual launch, for the kernels' live launch durations
    dt, rep, X = run(args.prec, args.steps, args.warmup, False)
    dt_prof, _, _ = run(args.prec, args.steps, 1, True)
    upd = spd.profile_query(spd.K_UPDATE)
    res = spd.profile_query(spd.K_RESIDUAL)
    kernels = kernel_summary(spd, args.prec)
    log(f"{args.prec}: {dt * 1e3:.2f} ms/solve ({dt_prof * 1e3:.2f} with kernel events), iters "
        f"{rep.iters_low}/{rep.iters_high}, eta {rep.eta:.2e}, status {rep.status}, update kernel {upd[0]} "
        f"launches {upd[1]:.2f} ms")
    fwd = float((X - Xt).abs().max() / Xt.abs().max())
    fwd_bound = 10 * cond * 2.0 ** -53

    fp64 = None
    if not args.no_fp64:
        dt64, rep64, X64 = run("fp64", args.steps, max(1, args.warmup), False)
        fwd64 = float((X64 - Xt).abs().max() / Xt.abs().max())
        # the binary64 path's own kernels (one evented solve): where its update stands against its peak
        run("fp64", 1, 0, True)
        fp64 = {"ms_per_step": dt64 * 1e3, "value": algo_flops(n, m) / dt64 / 1e12,
                "iters": [rep64.iters_low, rep64.iters_high], "eta": rep64.eta, "fwd_err": fwd64,
                "status": rep64.status, "kernels": kernel_summary(spd, "fp64")}
        log(f"fp64: {dt64 * 1e3:.2f} ms/solve, eta {rep64.eta:.2e}")

    external = None if (args.no_external or cov) else external_fp64_leg(args, torch, A, B, Xt)

    # the binary16 factor on a system of the same recipe at cond 1e2, where
    # cond u16 << 1 (configuration: the half-precision path at this size)
    half = None
    A16 = B16 = None
    if not args.no_half and not cov and args.prec == "fp32":
        A16 = spdgen.logspaced(n, args.half_cond, sg + 2, backend="torch", device="cuda")
        X16t = spdgen.rhs(n, m, sx + 2, backend="torch", device="cuda")
        B16 = spdgen.accurate_product(A16, X16t)
        Asave, Bsave = A, B
        A, B = A16, B16
        dt16, rep16, X16 = run("fp16", args.steps, args.warmup, False)
        dt16p, _, _ = run("fp16", args.steps, 1, True)
        k16 = kernel_summary(spd, "fp16")
        dt16_64, rep16_64, _ = run("fp64", args.steps, max(1, args.warmup), False) if not args.no_fp64 else (None, None, None)
        A, B = Asave, Bsave
        fwd16 = float((X16 - X16t).abs().max() / X16t.abs().max())
        half = {"workload": f"dense SPD, n={n}, cond={args.half_cond:g} (same recipe), {m} RHS, fp16 factor "
                            f"(equilibrated, mu = 4096) + binary64 refinement",
                "ms_per_step": dt16 * 1e3, "value": algo_flops(n, m) / dt16 / 1e12,
                "timed_with_events_ms_per_step": dt16p * 1e3,
                "accuracy": {"status": rep16.status, "prec_used": spd.PREC_NAME[rep16.prec_used],
                             "iters": [rep16.iters_low, rep16.iters_high], "eta": rep16.eta, "fwd_err_vs_xtrue": fwd16,
                             "fwd_bound_10cond_u": 10 * args.half_cond * 2.0 ** -53},
                "fp64_same_system_ms": dt16_64 * 1e3 if dt16_64 else None,
                "speedup_vs_fp64": (dt16_64 / dt16) if dt16_64 else None,
                "kernels": k16}
        log(f"fp16 (cond {args.half_cond:g}): {dt16 * 1e3:.2f} ms/solve, iters {rep16.iters_low}/{rep16.iters_high}, "
            f"fp64 {dt16_64 * 1e3 if dt16_64 else float('nan'):.2f} ms")

    energy = None
    if not args.no_energy and not cov and args.prec == "fp32":
        try:
            systems = [("fp32+IR", "fp32", A, B, algo_flops(n, m)), ("fp64", "fp64", A, B, algo_flops(n, m))]
            if A16 is not None:
                systems.insert(1, (f"fp16+IR cond {args.half_cond:g}", "fp16", A16, B16, algo_flops(n, m)))
            energy = energy_leg(args, spd, torch, systems, args.energy_window)
        except Exception as e:  # no power telemetry on this host
            energy = {"error": f"{type(e).__name__}: {e}"}
    del A16, B16

    batched = None if args.no_batched else batched_leg(args, spd, spdgen, torch)

    cpu = None
    ocheck = None
    if not args.no_cpu_baseline:
        cpu, ocheck = cpu_baseline_leg(args, A, X, B, rows_check=n <= 32768)

    launches, ms, fl, by = upd
    sched = None
    if args.prec in tuned:
        sched = {k: tuned[args.prec][k] for k in ("group", "upd_slots", "small_tiles")}
    traffic = None if cov or n != 16384 or sched is None else measured_traffic(args.prec, sched)
    traffic_input = None
    if traffic is not None:
        traffic, traffic_input = traffic
    achieved = fl / ms / 1e9 if ms > 0 else 0.0  # TFLOP/s
    peak = PEAK_TFLOPS[args.prec]
    out = {
        "metric": ("time to FP64-accurate solve & eff. TFLOP/s: mixed vs FP64 Cholesky, n=16384" if not cov else
                   f"time to FP64-accurate solve & eff. TFLOP/s: mixed vs FP64 Cholesky, covariance d={args.decay}, "
                   f"n={n}, m={m}"),
        "value": algo_flops(n, m) / dt / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "fp32" else f"{args.prec}+f32+f64",
        "data": "synthetic",
        "config": ({"workload": f"dense SPD A X = B, n={n}, cond={cond:g} (log-spaced eigenvalues, random "
                                f"orthogonal Q), {m} RHS, {args.prec} factor + binary64 refinement",
                    "n": n, "nrhs": m, "cond": cond, "prec": args.prec} if not cov else
                   {"workload": f"model covariance matrix (Section 4), d={args.decay}, n={n}, {m} RHS, "
                                f"{args.prec} factor + binary64 refinement",
                    "n": n, "nrhs": m, "decay": args.decay, "cond_bound": cond, "prec": args.prec}),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic, "traffic_input": traffic_input,
                     "kernel": ("k_syrk_update_f32 (a group's trailing update, 128- or 64-row tiles)"
                                if args.prec == "fp32" else (
                                    "k_syrk_update_h256 / k_syrk_update_h (a group's trailing update, "
                                    "binary16/bfloat16 operands)" if args.prec in ("fp16", "bf16")
                                    else "k_syrk_update<double>")),
                     "launches": launches, "avg_launch_ms": ms / max(launches, 1),
                     "timed_with_events_ms_per_step": dt_prof * 1e3,
                     "flops_per_launch": fl / max(launches, 1),
                     "algorithmic_bytes_per_launch": by / max(launches, 1)},
        "kernels": kernels,
        "cpu_baseline": cpu,
        "accuracy": {"status": rep.status, "iters": [rep.iters_low, rep.iters_high], "eta": rep.eta,
                     "fwd_err_vs_xtrue": fwd, "fwd_bound_10cond_u": fwd_bound, "oracle_rows": ocheck},
        "fp64_baseline": fp64,
        "speedup_vs_fp64": (fp64["ms_per_step"] / (dt * 1e3)) if fp64 else None,
        "external_fp64_reference": external,
        "autotune": tuned or None,
        "tune_cache": tune_source,
        "fp16_leg": half,
        "energy": energy,
        "batched": batched,
        "residual_kernel": {"launches": res[0], "avg_ms": res[1] / max(res[0], 1),
                            "achieved_GBs": (res[3] / res[1] / 1e6) if res[1] > 0 else None,
                            "hbm_peak_GBs": HBM_PEAK_GBS},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
