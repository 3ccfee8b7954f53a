"""Reference low-precision encodings used by the precision form.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written from the published definitions, with exact FP64 arithmetic on FP32
inputs:
  * bfloat16: the upper 16 bits of an IEEE binary32 value, rounded to
    nearest-even on the 16 dropped bits.
  * FP8 E4M3 in the OCP 8-bit floating point specification ("fn": 4 exponent
    bits with bias 7, 3 mantissa bits, no infinities, S.1111.111 is NaN, so
    the largest finite magnitude is 1.75 * 2^8 = 448; exponent field 0 holds
    subnormals m/8 * 2^-6).  Rounding is to nearest-even; magnitudes above 448
    saturate to 448.
  * Per-tensor scale for FP8: scale = amax / 448 (binary32 division), codes
    are e4m3(x / scale) with the division done in binary32, and a stored code
    c stands for value(c) * scale.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_bits(x32: np.ndarray) -> np.ndarray:
    """uint16 bfloat16 codes of float32 input, round-to-nearest-even."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) & 0xFFFF
    return r.astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """FP64 values of bfloat16 codes (exact)."""
    u = (np.asarray(bits, dtype=np.uint32) << 16).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def fp8_scale(x32: np.ndarray) -> np.float32:
    """Per-tensor scale amax / 448 in binary32; 1 for an all-zero tensor."""
    amax = np.float32(np.max(np.abs(np.asarray(x32, dtype=np.float32)))) if np.size(x32) else np.float32(0)
    if amax == 0:
        return np.float32(1.0)
    return np.float32(amax / np.float32(E4M3_MAX))


def e4m3_bits(y32: np.ndarray) -> np.ndarray:
    """uint8 E4M3 codes of float32 values (RNE, saturating at 448)."""
    y = np.asarray(y32, dtype=np.float32).astype(np.float64)
    sign = (y < 0) | ((y == 0) & np.signbit(y))
    a = np.abs(y)
    code = np.zeros(a.shape, dtype=np.int64)
    sat = a >= E4M3_MAX
    normal = (a >= 2.0 ** -6) & ~sat
    sub = (a < 2.0 ** -6)
    # subnormals: m = RNE(a / 2^-9), m == 8 is the smallest normal (E=1, m=0)
    ms = np.rint(a[sub] * 2.0 ** 9).astype(np.int64)
    code[sub] = ms  # E field 0 plus mantissa; ms == 8 encodes E=1, m=0 exactly
    # normals: a = 2^e (1 + f), mantissa RNE(f * 8), carry into the exponent
    an = a[normal]
    e = np.floor(np.log2(an)).astype(np.int64)
    # guard against log2 rounding at exact powers of two
    e = np.where(2.0 ** e > an, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= an, e + 1, e)
    m = np.rint((an / 2.0 ** e - 1.0) * 8.0).astype(np.int64)
    carry = m == 8
    e = np.where(carry, e + 1, e)
    m = np.where(carry, 0, m)
    E = e + 7
    c = (E << 3) | m
    c = np.where(c > 0x7E, 0x7E, c)  # 0x7E = 448; never emit the NaN code
    code[normal] = c
    code[sat] = 0x7E
    code = code | (sign.astype(np.int64) << 7)
    return code.astype(np.uint8)


def e4m3_value(bits: np.ndarray) -> np.ndarray:
    """FP64 values of E4M3 codes (exact; the NaN code maps to NaN)."""
    b = np.asarray(bits, dtype=np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    E = (b >> 3) & 0xF
    m = (b & 7).astype(np.float64)
    val = np.where(E == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (E - 7))
    val = np.where((E == 15) & ((b & 7) == 7), np.nan, val)
    return s * val


def quantize_fp8(x32: np.ndarray):
    """(codes, scale): codes = e4m3(x / scale) with the division in binary32."""
    x = np.asarray(x32, dtype=np.float32)
    scale = fp8_scale(x)
    y = (x / scale).astype(np.float32)
    return e4m3_bits(y), scale


def dequantize_fp8(codes: np.ndarray, scale) -> np.ndarray:
    return e4m3_value(codes) * float(np.float32(scale))
