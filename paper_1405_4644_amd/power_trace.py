"""Phase-resolved power and energy of a solve on one MI355X: the analogue of
the paper's power diagrams (Fig. 3(a) for Cholesky with refinement, Fig. 4
for CG with refinement) and of Table 2's time / average power / energy
columns, measured on the GPU instead of the whole blade.

A sampler thread reads the GPU's socket power and energy accumulator every
`period` seconds through amdsmi (read-only queries).  The device publishes
both about once per second, shorter than most phases here, so each phase is
executed repeatedly for at least `--window` seconds (after a device
synchronisation on both ends) and its steady-state power is the energy
accumulated between the first and the last publication inside that window
divided by the time between them; a phase's energy per execution is that
power times its own duration.  The amdsmi device is matched to torch's
device 0 by PCI address, so another GPU of the same host is never read.

    python -m paper_1405_4644_amd.power_trace --solver cholesky --nrhs 32 --decay 1
    python -m paper_1405_4644_amd.power_trace --solver cg --band 16 --nrhs 1 --decay 1 --out trace.json

Prints one JSON line: per phase the duration of one execution, its energy,
the average and peak power; the idle power; and, with --out, the whole
sample trace.
"""
from __future__ import annotations

import argparse
import json
import threading
import time


def summarize(samples, marks):
    """Per-phase figures from the trace.

    samples: [(t, watts, joules)] in time order (joules: the energy
    accumulator, None where unreadable); marks: [(name, t_start, t_end,
    executions)].  Average power: energy between the first and the last
    accumulator publication (a change of its value) inside the phase over the
    time between them; without two publications, the mean of the distinct
    power readings inside the phase.  Energy per execution = average power x
    the mean duration of one execution; peak = the largest reading."""
    out = []
    for name, t0, t1, reps in marks:
        inside = [(t, w, e) for t, w, e in samples if t0 <= t <= t1]
        pubs, last = [], None
        for t, w, e in samples:
            if e is not None and e != last:
                if t0 <= t <= t1 and last is not None:
                    pubs.append((t, e))
                last = e
        avg = None
        if len(pubs) >= 2 and pubs[-1][0] > pubs[0][0]:
            avg = (pubs[-1][1] - pubs[0][1]) / (pubs[-1][0] - pubs[0][0])
        else:
            readings, prev = [], None
            for _, w, _ in inside:
                if w != prev:
                    readings.append(w)
                prev = w
            avg = sum(readings) / len(readings) if readings else None
        one = (t1 - t0) / max(reps, 1)
        out.append({"phase": name, "seconds": one, "executions": reps, "window_seconds": t1 - t0,
                    "avg_watts": avg, "joules": avg * one if avg is not None else None,
                    "peak_watts": max((w for _, w, _ in inside), default=None),
                    "energy_publications": len(pubs)})
    return out


class PowerMonitor:
    """Samples socket power of the GPU behind torch device 0."""

    def __init__(self, period: float = 0.002):
        import amdsmi
        import torch
        self._smi = amdsmi
        amdsmi.amdsmi_init()
        prop = torch.cuda.get_device_properties(0)
        want = (int(prop.pci_domain_id), int(prop.pci_bus_id), int(prop.pci_device_id))
        self.h = None
        for h in amdsmi.amdsmi_get_processor_handles():
            bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)  # "dddd:bb:dd.f"
            dom, bus, rest = bdf.split(":")
            if (int(dom, 16), int(bus, 16), int(rest.split(".")[0], 16)) == want:
                self.h = h
                break
        if self.h is None:
            raise RuntimeError(f"no amdsmi device with PCI address {want}")
        self.period = period
        self.samples: list[tuple[float, float, float | None]] = []
        self.marks: list[tuple[str, float, float, int]] = []
        self._stop = threading.Event()
        self._thr = None
        self._t0 = time.perf_counter()

    def power(self) -> float:
        info = self._smi.amdsmi_get_power_info(self.h)
        for key in ("current_socket_power", "average_socket_power", "socket_power"):
            v = info.get(key)
            if isinstance(v, (int, float)) and v > 0:
                return float(v)
        raise RuntimeError("no socket power reading")

    def joules(self) -> float | None:
        try:
            e = self._smi.amdsmi_get_energy_count(self.h)
            return e["energy_accumulator"] * e["counter_resolution"] * 1e-6
        except Exception:
            return None

    def _run(self):
        while not self._stop.is_set():
            try:
                self.samples.append((time.perf_counter() - self._t0, self.power(), self.joules()))
            except Exception:
                pass
            time.sleep(self.period)

    def start(self):
        self._thr = threading.Thread(target=self._run, daemon=True)
        self._thr.start()

    def phase(self, name, fn, window: float = 0.0, reset=None):
        """Run fn() as one phase, repeated (reset() before each repeat) until
        `window` seconds have passed; synchronise before and after and record
        the span and the number of executions.  Returns the first result."""
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter() - self._t0
        r = fn()
        reps = 1
        torch.cuda.synchronize()
        while time.perf_counter() - self._t0 - t0 < window:
            if reset:
                reset()
            fn()
            reps += 1
            torch.cuda.synchronize()
        self.marks.append((name, t0, time.perf_counter() - self._t0, reps))
        return r

    def stop(self):
        self._stop.set()
        if self._thr:
            self._thr.join()
        try:
            self._smi.amdsmi_shut_down()
        except Exception:
            pass

    def report(self):
        return summarize(self.samples, self.marks)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--solver", choices=["cholesky", "cg"], default="cholesky")
    ap.add_argument("--n", type=int, default=70000)
    ap.add_argument("--decay", type=int, choices=[1, 2, 4], default=1)
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp16", "bf16", "fp64"])
    ap.add_argument("--band", type=int, default=-1, help="--solver cg: half-bandwidth (-1 dense)")
    ap.add_argument("--window", type=float, default=4.0, help="seconds each phase (and idle) is repeated for")
    ap.add_argument("--period", type=float, default=0.002)
    ap.add_argument("--out", default=None, help="write the whole trace (JSON) here")
    a = ap.parse_args(argv)

    import torch

    import paper_1405_4644_amd as spd
    import spdgen

    spd.load()
    n, m = a.n, a.nrhs
    A = spdgen.covariance(n, a.decay, backend="torch", device="cuda")
    _, sx = spdgen.seeds(5, a.decay)
    Xt = spdgen.rhs(n, m, sx, backend="torch", device="cuda")
    B = spdgen.accurate_product(A, Xt)
    # one untimed solve first (code loading, workspace allocation)
    if a.solver == "cholesky":
        spd.posv(A, B, prec=a.prec)
    else:
        H0 = spd.cg_prepare(A, half_band=a.band)
        spd.cg_refine(H0, A, B)
        H0.close()
    torch.cuda.synchronize()

    mon = PowerMonitor(a.period)
    mon.start()
    W = a.window
    mon.phase("idle", lambda: time.sleep(0.05), W)
    if a.solver == "cholesky":
        F = spd.Factor()
        mon.phase("factor (Algorithm 1, low-precision Cholesky)", lambda: spd.factor(A, prec=a.prec, F=F), W)
        X0 = mon.phase("first solve", lambda: spd.solve(F, B), W)
        X = torch.empty_like(X0)
        X.copy_(X0)
        rep = mon.phase("refinement", lambda: spd.refine(F, A, B, X), W, reset=lambda: X.copy_(X0))
        F.close()
    else:
        H = spd.CG()
        mon.phase("operator A~ (binary32)", lambda: spd.cg_prepare(A, half_band=a.band, H=H), W)
        X = torch.zeros_like(B)
        X, rep = mon.phase("CG with refinement (Algorithm 2)", lambda: spd.cg_refine(H, A, B, X), W,
                           reset=lambda: X.zero_())
        H.close()
    mon.stop()
    phases = mon.report()
    idle = next(p for p in phases if p["phase"] == "idle")
    work = [p for p in phases if p["phase"] != "idle"]
    tot_s = sum(p["seconds"] for p in work)
    tot_j = sum(p["joules"] for p in work if p["joules"] is not None)
    # net of idle: the energy the solve adds above the idle draw
    out = {"solver": a.solver, "n": n, "nrhs": m, "decay": a.decay,
           "prec": a.prec if a.solver == "cholesky" else "fp32 operator + fp64",
           "band": a.band if a.solver == "cg" else None,
           "status": rep.status, "iters": [rep.iters_low, rep.iters_high], "eta": rep.eta,
           "idle_watts": idle["avg_watts"], "phases": work, "seconds": tot_s, "joules": tot_j,
           "avg_watts": tot_j / tot_s if tot_s > 0 else None,
           "joules_above_idle": (tot_j - idle["avg_watts"] * tot_s) if idle["avg_watts"] is not None else None,
           "peak_watts": max((p["peak_watts"] or 0.0) for p in work)}
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": out, "samples": mon.samples, "marks": mon.marks}, f)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
