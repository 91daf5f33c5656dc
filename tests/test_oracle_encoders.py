"""Pins for the storage encoders of the oracle against independent
implementations (numpy's C binary16 cast, torch's float8_e4m3fn cast) and the
format definitions' fixed points."""
import numpy as np
import pytest
import torch

from oracle import encoders

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _specials32():
    vals = [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.0, 65520.0, 70000.0, 2.0 ** -14, 2.0 ** -24,
            2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -15 + 2.0 ** -25, 0.1, 1.0 / 3.0, np.inf, -np.inf, np.nan]
    # binary16 midpoints in several binades (ties to even)
    for e in (-14, -3, 0, 5, 14):
        q = 2.0 ** (e - 10)
        for m in (0, 1, 2, 511, 1022):
            vals.append((1.0 + m / 1024.0) * 2.0 ** e + q / 2)
    return np.array(vals, dtype=np.float32)


def test_f16_bits_match_numpy_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        _specials32(),
        rng.standard_normal(200000).astype(np.float32) * 10,
        (rng.standard_normal(50000) * 1e-5).astype(np.float32),
        rng.uniform(-7e4, 7e4, 50000).astype(np.float32),
    ])
    ref = x.astype(np.float16).view(np.uint16)
    got = encoders.f16_bits(x)
    nan = np.isnan(x)
    assert np.array_equal(got[~nan], ref[~nan])
    assert np.all((got[nan] & 0x7C00) == 0x7C00) and np.all(got[nan] & 0x3FF)


def test_f16_value_matches_numpy():
    bits = np.arange(0, 65536, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = encoders.f16_value(bits)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_e4m3_fixed_points():
    v = encoders.e4m3_value
    assert v(0x00) == 0.0
    assert v(0x01) == 2.0 ** -9          # smallest subnormal
    assert v(0x07) == 7 * 2.0 ** -9      # largest subnormal
    assert v(0x08) == 2.0 ** -6          # smallest normal
    assert v(0x38) == 1.0
    assert v(0x7E) == 448.0              # largest finite
    assert np.isnan(v(0x7F)) and np.isnan(v(0xFF))
    assert v(0xB8) == -1.0
    mags = v(np.arange(0, 127))
    assert np.all(np.diff(mags) > 0)     # strictly increasing grid


def test_e4m3_decode_matches_torch():
    codes = torch.arange(0, 256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = encoders.e4m3_value(np.arange(256))
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(1)
    grid = encoders.e4m3_value(np.arange(0, 127))
    mids = (grid[1:] + grid[:-1]) / 2
    x = np.concatenate([
        rng.uniform(-448, 448, 200000), rng.standard_normal(100000) * 0.01,
        grid, -grid, mids, -mids, mids * (1 + 1e-7), mids * (1 - 1e-7),
    ]).astype(np.float32)
    x = x[np.abs(x) <= 448]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = encoders.e4m3_encode(x)
    # torch keeps the sign of zero; so do we
    assert np.array_equal(got, ref)


def test_e4m3_saturates_and_nan():
    x = np.array([448.0, 449.0, 464.0, 1e6, np.inf, -500.0, -np.inf, np.nan], dtype=np.float32)
    got = encoders.e4m3_encode(x)
    assert list(got[:5]) == [0x7E] * 5
    assert list(got[5:7]) == [0xFE, 0xFE]
    assert got[7] & 0x7F == 0x7F


def test_e4m3_ties_to_even():
    # midpoint between 1.0 (0x38, even mantissa) and 1.125 (0x39) goes to 1.0;
    # midpoint between 1.125 and 1.25 (0x3A) goes to 1.25
    got = encoders.e4m3_encode(np.array([1.0625, 1.1875, 2.0 ** -10, 3 * 2.0 ** -10], dtype=np.float32))
    assert list(got) == [0x38, 0x3A, 0x00, 0x02]


def test_brick_quantiser_range_and_degenerate():
    rng = np.random.default_rng(2)
    v = (rng.standard_normal(10000) * 3 + 1).astype(np.float32)
    s, o = encoders.brick_scale_offset(float(v.min()), float(v.max()))
    codes = encoders.fp8_encode_brick(v, s, o)
    dec = encoders.fp8_decode_brick(codes, s, o)
    # extremes map to +-448 and decode within the top-binade step
    assert encoders.e4m3_value(codes[np.argmax(v)]) == 448.0
    assert encoders.e4m3_value(codes[np.argmin(v)]) == -448.0
    rel = np.abs(dec - v) / np.maximum(np.abs(v - o), 2.0 ** -6 * s)
    assert np.max(rel) <= 2.0 ** -4 + 1e-6         # 3-bit mantissa: half-ulp <= 1/16
    s1, o1 = encoders.brick_scale_offset(2.5, 2.5)
    assert s1 == 1.0 and o1 == np.float32(2.5)
    c = encoders.fp8_encode_brick(np.full(5, 2.5, np.float32), s1, o1)
    assert np.all(encoders.fp8_decode_brick(c, s1, o1) == 2.5)
