"""Pins of the oracle's BF16 / FP8-E4M3 encoders against the published
formats: exhaustive code round trips, hand-computed boundary values, and
torch's own (independent) conversions on random data."""
import numpy as np
import pytest
import torch

from oracle import quant


def test_e4m3_decode_table_boundaries():
    # OCP E4M3: max finite 448 (0x7E), min normal 2^-6 (0x08), min subnormal 2^-9 (0x01)
    assert quant.e4m3_value(np.array([0x7E]))[0] == 448.0
    assert quant.e4m3_value(np.array([0x08]))[0] == 2.0 ** -6
    assert quant.e4m3_value(np.array([0x01]))[0] == 2.0 ** -9
    assert quant.e4m3_value(np.array([0x38]))[0] == 1.0
    assert quant.e4m3_value(np.array([0xB8]))[0] == -1.0
    assert np.isnan(quant.e4m3_value(np.array([0x7F]))[0])


def test_e4m3_roundtrip_all_codes():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = quant.e4m3_value(codes).astype(np.float32)
    back = quant.e4m3_bits(vals)
    # -0 and +0 both decode to 0; the sign of zero is kept
    np.testing.assert_array_equal(back, codes)


def test_e4m3_rounding_and_saturation():
    cases = {
        1.0 + 1 / 16: 0x38,      # tie between 1 and 1.125 -> even mantissa (1.0)
        1.0 + 3 / 16: 0x3A,      # tie between 1.125 and 1.25 -> even (1.25)
        460.0: 0x7E, 1e6: 0x7E,  # saturation at 448
        2.0 ** -10: 0x00,        # tie between 0 and 2^-9 -> even (0)
        3 * 2.0 ** -10: 0x02,    # tie between 2^-9 and 2*2^-9 -> even (2)
        15 * 2.0 ** -10: 0x08,   # rounds up into the smallest normal
    }
    for v, c in cases.items():
        assert quant.e4m3_bits(np.array([v], dtype=np.float32))[0] == c, v
        assert quant.e4m3_bits(np.array([-v], dtype=np.float32))[0] == (c | 0x80), v


def test_e4m3_matches_torch_in_range():
    x = (np.random.default_rng(3).standard_normal(200000) * 60).astype(np.float32)
    x = np.clip(x, -448, 448)
    ours = quant.e4m3_bits(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_bf16_matches_torch():
    x = np.random.default_rng(4).standard_normal(200000).astype(np.float32) * 1e3
    ours = quant.bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_fp8_scale_and_dequant_error():
    x = np.random.default_rng(5).standard_normal(10000).astype(np.float32)
    codes, s = quant.quantize_fp8(x)
    assert s == np.float32(np.float32(np.abs(x).max()) / np.float32(448))
    y = quant.dequantize_fp8(codes, s)
    # relative spacing of e4m3 normals is 2^-3: RNE error <= 2^-4 relative
    big = np.abs(x) > 2.0 ** -6 * s
    assert np.all(np.abs(y[big] - x[big]) <= np.abs(x[big]) * 2.0 ** -4 * (1 + 1e-6))
