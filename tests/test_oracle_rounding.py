"""Pins for the oracle's binary32 -> binary16 / bfloat16 round-to-nearest-even.

Checked against the formats' own definitions (every representable value is a
fixed point, midpoints go to the even neighbour) and, independently, against
numpy's float16 and torch's bfloat16 conversions.
"""
import numpy as np
import pytest


def _f16_values():
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    return bits.view(np.float16).astype(np.float32)


def _bf16_values():
    bits = (np.arange(1 << 16, dtype=np.uint32) << 16).astype(np.uint32)
    return bits.view(np.float32)


def test_f16_fixed_points_exhaustive(orc):
    v = _f16_values()
    v = v[np.isfinite(v)]
    got = np.array([orc.rne_f16(x) for x in v], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), v.view(np.uint32))


def test_bf16_fixed_points_exhaustive(orc):
    v = _bf16_values()
    v = v[np.isfinite(v)]
    got = np.array([orc.rne_bf16(x) for x in v], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), v.view(np.uint32))


def test_f16_ties_to_even(orc):
    v = np.sort(np.unique(_f16_values()[np.isfinite(_f16_values())]))
    v = v[(v > 0)]
    lo, hi = v[:-1].astype(np.float64), v[1:].astype(np.float64)
    mid = ((lo + hi) / 2).astype(np.float32)
    assert np.all(mid.astype(np.float64) == (lo + hi) / 2)  # midpoints are exact in binary32
    got = np.array([orc.rne_f16(x) for x in mid[::37]], dtype=np.float32)
    lo16 = lo[::37].astype(np.float16)
    hi16 = hi[::37].astype(np.float16)
    lo_even = (lo16.view(np.uint16) & 1) == 0
    want = np.where(lo_even, lo16, hi16).astype(np.float32)
    assert np.array_equal(got, want)
    # overflow boundary: 65520 is the midpoint between 65504 and 2^16 -> inf
    assert orc.rne_f16(65519.996) == 65504.0
    assert np.isinf(orc.rne_f16(65520.0))
    assert orc.rne_f16(-65520.0) == -np.inf


def test_f16_against_numpy_random(orc):
    rng = np.random.Generator(np.random.PCG64(1))
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5, 20000)).astype(np.float32)
    got = np.array([orc.rne_f16(v) for v in x], dtype=np.float32)
    want = x.astype(np.float16).astype(np.float32)
    assert np.array_equal(got, want)


def test_bf16_against_torch_random(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(2))
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000)).astype(np.float32)
    got = np.array([orc.rne_bf16(v) for v in x], dtype=np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got, want)


def test_bf16_ties_to_even(orc):
    # 1 + 2^-8 is the midpoint between 1 and 1 + 2^-7: ties to even -> 1
    assert orc.rne_bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3*2^-8 is the midpoint between 1+2^-7 (odd) and 1+2^-6 (even) -> 1+2^-6
    assert orc.rne_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert np.isnan(orc.rne_bf16(float("nan")))
