"""FP16C, a 16-bit storage format for shifted populations (test infrastructure).

The paper's mixed-precision section (Sec. IV.A, second group) cites a
customised half-precision format, FP16C, that halves the rounding error of
IEEE binary16 when the stored values are the shifted populations of
Eq. shift_f.  The paper does not print its layout; it is read here as the
format with one more significand bit than binary16:
  bit 15        sign
  bits 14..11   exponent field e (4 bits, bias 15)
  bits 10..0    significand field m (11 bits)
  value         (-1)^s (1 + m / 2^11) 2^(e - 15)   for e >= 1   (normal, 2^-14 <= |v| < 2)
                (-1)^s  m 2^-25                      for e == 0   (subnormal)
There is no infinity or NaN: encoding saturates at the largest magnitude
2 - 2^-11.  Encoding rounds to the nearest value, ties to the even code.

Everything here follows from that definition (float64 arithmetic, exact for
these magnitudes); nothing is shared with the device encoder.
"""
from __future__ import annotations

import numpy as np

BIAS = 15
MANT_BITS = 11
MAX_VALUE = 2.0 - 2.0 ** -MANT_BITS
MIN_NORMAL = 2.0 ** (1 - BIAS)
SUB_STEP = 2.0 ** (1 - BIAS - MANT_BITS)     # 2^-25


def decode(codes):
    """float64 values of uint16 codes."""
    h = np.asarray(codes).astype(np.int64) & 0xFFFF
    e = (h >> MANT_BITS) & 0xF
    m = h & ((1 << MANT_BITS) - 1)
    mag = np.where(e == 0, m * SUB_STEP, (1.0 + m / 2.0 ** MANT_BITS) * np.exp2(e - BIAS))
    return np.where(h & 0x8000, -mag, mag)


def _grid(a):
    """Spacing of representable magnitudes around a >= 0 (the spacing of the
    binade a lies in, or the subnormal step below 2^-14)."""
    mant, ex = np.frexp(np.where(a > 0, a, 1.0))      # a = mant 2^ex, mant in [0.5, 1)
    top = np.maximum(ex - 1, 1 - BIAS)                # exponent of the binade
    return np.exp2(top - MANT_BITS)


def encode(x):
    """uint16 codes of the nearest FP16C values of x (float64 or float32),
    ties to the even code, magnitudes beyond the largest value saturated."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    step = _grid(a)
    n = np.rint(a / step)                             # ties to even multiple of the step
    v = np.minimum(n * step, MAX_VALUE)
    # the code of the representable magnitude v
    mant, ex = np.frexp(np.where(v > 0, v, 1.0))
    e = np.where(v >= MIN_NORMAL, ex - 1 + BIAS, 0)
    m = np.where(e == 0, np.rint(v / SUB_STEP),
                 np.rint((v / np.exp2(e - BIAS) - 1.0) * 2.0 ** MANT_BITS))
    code = (e.astype(np.int64) << MANT_BITS) | m.astype(np.int64)
    return (code | np.where(np.signbit(x), 0x8000, 0)).astype(np.uint16)


def round_fp16c(x):
    """x rounded to FP16C and back, as float64."""
    return decode(encode(x))


__all__ = ["decode", "encode", "round_fp16c", "MAX_VALUE", "MIN_NORMAL", "SUB_STEP"]
