"""The power-trace harness (phase-resolved power and energy, the analogue of
Figs. 3(a) and 4): its per-phase arithmetic on the CPU, and one traced solve
on the GPU when the GPU's power can be read."""
import pytest

from paper_1405_4644_amd.power_trace import summarize


def test_summary_uses_energy_publications():
    # accumulator published once a second: 100 J/s in phase a, 300 J/s in b
    samples = []
    e = 0.0
    for k in range(0, 81):
        t = k * 0.05
        if k % 20 == 0 and k > 0:
            e += 100.0 if t <= 2.0 else 300.0
        samples.append((t, 100.0 if t <= 2.0 else 300.0, e))
    out = summarize(samples, [("a", 0.0, 2.0, 4), ("b", 2.0, 4.0, 1)])
    a, b = out
    assert a["energy_publications"] == 2 and a["avg_watts"] == pytest.approx(100.0)
    assert a["seconds"] == pytest.approx(0.5) and a["joules"] == pytest.approx(50.0)
    assert b["avg_watts"] == pytest.approx(300.0) and b["joules"] == pytest.approx(600.0)
    assert b["peak_watts"] == 300.0


def test_summary_without_counter_uses_distinct_readings():
    samples = [(0.0, 100.0, None), (0.4, 100.0, None), (0.5, 200.0, None), (0.9, 200.0, None), (1.0, 600.0, None)]
    out = summarize(samples, [("x", 0.0, 1.0, 2)])
    assert out[0]["avg_watts"] == pytest.approx(300.0) and out[0]["joules"] == pytest.approx(150.0)


def test_empty_phase():
    out = summarize([], [("x", 0.0, 0.0, 1)])
    assert out[0]["avg_watts"] is None and out[0]["joules"] is None


@pytest.mark.gpu
def test_traced_solve(spd):
    import torch

    import spdgen
    from paper_1405_4644_amd.power_trace import PowerMonitor
    try:
        mon = PowerMonitor(0.002)
        mon.power()
    except Exception as e:  # no readable power sensor for this device
        pytest.skip(f"GPU power not readable: {e}")
    n = 4096
    A = spdgen.covariance(n, 1, backend="torch", device="cuda")
    B = spdgen.rhs(n, 4, 3, backend="torch", device="cuda")
    mon.start()
    F = mon.phase("factor", lambda: spd.factor(A, prec="fp32")[0], 1.5)
    X = mon.phase("solve", lambda: spd.solve(F, B))
    rep = mon.phase("refine", lambda: spd.refine(F, A, B, X))
    mon.stop()
    torch.cuda.synchronize()
    assert rep.status == 0
    out = mon.report()
    assert [p["phase"] for p in out] == ["factor", "solve", "refine"]
    for p in out:
        assert p["seconds"] > 0
        assert p["joules"] is None or p["joules"] >= 0
    assert out[0]["executions"] > 1 and out[0]["avg_watts"] > 0
    assert len(mon.samples) > 0 and all(w > 0 for _, w, _ in mon.samples)
