"""Bit-exact GPU parity of the library's BF16 rounding kernels against the oracle: FP32 -> BF16
over every one of the 2^32 FP32 bit patterns, and FP64 -> BF16 (single rounding, the CP-ALS
factor store) on random values over the whole range, values beside every kind of rounding
midpoint, and the special values."""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_f32_to_bf16_every_bit_pattern(gpu):
    import paper_1809_09175_amd as spt
    for c in range((1 << 32) // CHUNK):
        lo = c * CHUNK
        _log(f"f32->bf16 patterns [{lo:#010x}, {lo + CHUNK:#010x})")
        start = lo - (1 << 32) if lo >= (1 << 31) else lo   # the same bits as int32
        x = torch.arange(start, start + CHUNK, dtype=torch.int32, device=gpu).view(torch.float32)
        got = spt.to_bf16(x).view(torch.int16).cpu().numpy().view(np.uint16)
        del x
        bits = np.arange(lo, lo + CHUNK, dtype=np.uint64).astype(np.uint32)
        ref = oracle.bf16_rne(bits)
        if not np.array_equal(got, ref):
            bad = np.nonzero(got != ref)[0][:5]
            raise AssertionError([(hex(int(bits[i])), hex(int(got[i])), hex(int(ref[i])))
                                  for i in bad])


def _f64_cases(rng, n):
    e = rng.integers(-160, 140, size=n)
    v = rng.random(n) * np.ldexp(1.0, e) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    # values at, just above and just below the midpoints between neighbouring BF16 values
    # (including the subnormal range and the step past the largest finite one)
    hi16 = rng.integers(0, 0x7F7F, size=n // 4, dtype=np.uint32)
    a = (hi16 << 16).view(np.float32).astype(np.float64)
    b = ((hi16 + 1) << 16).view(np.float32).astype(np.float64)
    mid = (a + b) / 2
    top = float(np.frombuffer(np.uint32(0x7F7F0000).tobytes(), np.float32)[0])
    mid_top = (top + 2.0 ** 128) / 2
    near = np.concatenate([mid, np.nextafter(mid, np.inf), np.nextafter(mid, -np.inf),
                           [mid_top, np.nextafter(mid_top, 0.0), np.nextafter(mid_top, np.inf)]])
    # FP32 values themselves, and doubles that an FP32 step would round onto a BF16 midpoint
    f32 = rng.integers(0, 1 << 32, size=n // 4, dtype=np.uint64).astype(np.uint32).view(np.float32)
    f32 = f32[np.isfinite(f32)].astype(np.float64)
    twice = mid * (1.0 + 2.0 ** -40)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 2.0 ** 128, -(2.0 ** 128),
                        np.finfo(np.float64).max, 5e-324, -5e-324, 2.0 ** -134, 2.0 ** -133,
                        2.0 ** -150, 2.0 ** -149, 2.0 ** -126, 1.0 + 2.0 ** -8 + 2.0 ** -30])
    return np.concatenate([v, near, -near, f32, twice, special])


def test_f64_to_bf16_matches_oracle(gpu):
    import paper_1809_09175_amd as spt
    rng = np.random.default_rng(61)
    v = _f64_cases(rng, 4_000_000)
    _log(f"f64->bf16 on {v.size} values")
    got = spt.to_bf16(torch.from_numpy(v).to(gpu)).view(torch.int16).cpu().numpy().view(np.uint16)
    ref = oracle.bf16_rne_f64(v)
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0][:5]
        raise AssertionError([(repr(float(v[i])), hex(int(got[i])), hex(int(ref[i]))) for i in bad])
    # the single rounding differs from rounding through FP32 on some of these inputs
    assert np.any(ref != oracle.bf16_rne(v.astype(np.float32)))
