"""Descriptor storage formats (input preparation, not matching arithmetic).

* BF16: round-to-nearest-even truncation of the FP32 bit pattern.
* FP8 E4M3FN (OCP): 1 sign, 4 exponent (bias 7), 3 mantissa bits, no
  infinities, max finite 448, subnormals down to 2**-9.  Each descriptor row
  gets an FP32 scale s = amax/448 and is stored as q = RNE_sat(d / s).
"""

import numpy as np

FP8_MAX = 448.0


def f32_to_bf16(x):
    """FP32 array -> uint16 BF16 bit patterns, round to nearest even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x)
    bias = ((u >> 16) & 1) + 0x7FFF
    r = ((u + bias) >> 16).astype(np.uint16)
    r[nan] = 0x7FC0
    return r


def bf16_to_f32(b):
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def _encode_e4m3(v):
    """FP32 values (already scaled) -> uint8 E4M3FN codes, RNE, saturating."""
    v = np.asarray(v, dtype=np.float64)
    sign = (v < 0) | ((v == 0) & np.signbit(v))
    a = np.minimum(np.abs(v), FP8_MAX)
    code = np.zeros(a.shape, dtype=np.int64)
    # subnormal range: a < 2**-6, step 2**-9 (np.rint rounds half to even)
    sub = a < 2.0 ** -6
    q = np.rint(a[sub] / 2.0 ** -9).astype(np.int64)  # 0..8; 8 == min normal
    code[sub] = q  # exp field 0 for q<8, q==8 encodes as exp 1 mant 0 == 8
    nrm = ~sub
    an = a[nrm]
    e = np.floor(np.log2(an)).astype(np.int64)
    # guard against log2 rounding at exact powers of two
    e = np.where(2.0 ** e > an, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= an, e + 1, e)
    mant = np.rint(an / 2.0 ** e * 8.0).astype(np.int64)  # 8..16
    carry = mant == 16
    e = np.where(carry, e + 1, e)
    mant = np.where(carry, 8, mant)
    ef = e + 7
    c = (ef << 3) | (mant - 8)
    c = np.minimum(c, 0x7E)  # 448 is the largest finite code (0x7E)
    code[nrm] = c
    return (code | (sign.astype(np.int64) << 7)).astype(np.uint8)


def fp8_e4m3_to_f32(c):
    c = np.asarray(c, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 7
    val = np.where(e == 0, m * 2.0 ** -9, (8 + m) * 2.0 ** (e - 7 - 3))
    val = np.where((e == 15) & (m == 7), np.nan, val)
    return (s * val).astype(np.float32)


def f32_to_fp8_e4m3(d):
    """Rows of FP32 descriptors -> (uint8 codes, FP32 per-row scale)."""
    d = np.ascontiguousarray(d, dtype=np.float32)
    amax = np.abs(d).max(axis=1)
    scale = (amax / np.float32(FP8_MAX)).astype(np.float32)
    scale = np.where(scale > 0, scale, np.float32(1.0)).astype(np.float32)
    scaled = (d / scale[:, None]).astype(np.float32)
    return _encode_e4m3(scaled), scale
