"""Reference conversions of FP32 values to BF16 and to OCP FP8 e4m3, written from
the formats' definitions, for checking the reduced-precision operands of the
distance product element by element.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
library imports this module.

Both conversions work the same way, by definition rather than by bit tricks:
every code of the target format is decoded to its exact value (FP64 holds all
of them exactly), and an input is mapped to the nearest representable value,
ties going to the code with an even significand (round to nearest even).

* BF16: 1 sign bit, 8 exponent bits (bias 127), 7 fraction bits; the same
  exponent range as FP32, with subnormals, infinities and NaNs.  Values beyond
  the largest finite BF16 by half an ulp or more round to infinity; a NaN stays
  a NaN (quiet, sign kept).
* OCP e4m3 ("E4M3FN"): 1 sign bit, 4 exponent bits (bias 7), 3 mantissa bits;
  subnormals with exponent field 0 (steps of 2^-9), no infinities, the single
  NaN code S.1111.111 and largest finite magnitude 448 (S.1111.110).  This
  library converts with saturation: magnitudes above 448, infinities included,
  become +-448; a NaN becomes the NaN code with its sign.
* Per-point scale of the FP8 operands: e is the largest integer with
  max_t |x_t| 2^e <= 448 (0 for a point without a finite non-zero element),
  limited to [-100, 100]; the point is stored as e4m3(x_t 2^e) with scale 2^-e.
"""
from __future__ import annotations

import numpy as np


def _bf16_table():
    """Exact values of the 32768 non-negative BF16 codes (NaN codes as NaN)."""
    codes = np.arange(1 << 15, dtype=np.int64)
    e = codes >> 7
    f = codes & 0x7F
    val = np.where(e == 0, f * 2.0 ** -133, (1.0 + f / 128.0) * np.exp2(e.astype(np.float64) - 127.0))
    val = np.where(e == 0xFF, np.where(f == 0, np.inf, np.nan), val)
    return val


def _e4m3_table():
    """Exact values of the 128 non-negative e4m3 codes (the NaN code as NaN)."""
    codes = np.arange(128, dtype=np.int64)
    e = codes >> 3
    m = codes & 7
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e.astype(np.float64) - 7.0))
    val = np.where(codes == 0x7F, np.nan, val)
    return val


_BF16 = _bf16_table()
_E4M3 = _e4m3_table()


def bf16_value(code: int) -> float:
    """The value of one BF16 code (16-bit pattern)."""
    v = _BF16[code & 0x7FFF]
    return -v if code & 0x8000 else v


def e4m3_value(code: int) -> float:
    """The value of one e4m3 code (8-bit pattern)."""
    v = _E4M3[code & 0x7F]
    return -v if code & 0x80 else v


def _nearest_even(a: np.ndarray, table: np.ndarray, top: int) -> np.ndarray:
    """Codes 0..top of `table` (ascending, exact values) nearest to the
    magnitudes `a` (finite, >= 0, at most table[top] + half its ulp), ties to
    the even code."""
    t = table[:top + 1]
    hi = np.searchsorted(t, a, side="left")          # first code with value >= a
    hi = np.minimum(hi, top)
    lo = np.maximum(hi - 1, 0)
    dlo = a - t[lo]
    dhi = t[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    return np.where(t[hi] == a, hi, code)


def to_bf16(x: np.ndarray) -> np.ndarray:
    """FP32 array -> BF16 codes (uint16), round to nearest even."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.int64)
    sign = (bits >> 31) << 15
    a = np.abs(x.astype(np.float64))
    out = np.zeros(x.shape, dtype=np.int64)
    top = 0x7F7F                                    # largest finite BF16
    big = a >= _BF16[top] + 2.0 ** (127 - 8)        # half an ulp above it, or more (or infinite)
    fin = np.isfinite(a) & ~big
    out[fin] = _nearest_even(a[fin], _BF16, top)
    out[big & ~np.isnan(a)] = 0x7F80
    nan = np.isnan(a)
    out[nan] = ((bits[nan] >> 16) & 0x7FFF) | 0x40
    return (out | sign).astype(np.uint16)


def to_e4m3(x: np.ndarray) -> np.ndarray:
    """FP32 (or FP64) array -> e4m3 codes (uint8), round to nearest even,
    saturating at +-448; NaN -> the NaN code."""
    x = np.asarray(x)
    a = np.abs(x.astype(np.float64))
    sign = np.signbit(x).astype(np.int64) << 7
    out = np.full(x.shape, 0x7E, dtype=np.int64)    # saturated magnitude 448
    inr = a <= 448.0
    out[inr] = _nearest_even(a[inr], _E4M3, 0x7E)
    out[np.isnan(a)] = 0x7F
    return (out | sign).astype(np.uint8)


def fp8_scale_exponent(row: np.ndarray) -> int:
    """Largest integer e with max|x| 2^e <= 448 (0 without a finite non-zero
    element), limited to [-100, 100]."""
    a = np.abs(np.asarray(row, dtype=np.float64))
    a = a[np.isfinite(a)]
    amax = float(a.max()) if a.size else 0.0
    if amax == 0.0:
        return 0
    e = int(np.floor(np.log2(448.0 / amax)))
    while np.ldexp(amax, e + 1) <= 448.0:
        e += 1
    while np.ldexp(amax, e) > 448.0:
        e -= 1
    return max(-100, min(100, e))


def quantize_fp8(X: np.ndarray):
    """Rows of X (n x d FP32) -> (codes n x d uint8, scales n float32 = 2^-e)."""
    X = np.asarray(X, dtype=np.float32)
    codes = np.empty(X.shape, np.uint8)
    scales = np.empty(X.shape[0], np.float32)
    for i in range(X.shape[0]):
        e = fp8_scale_exponent(X[i])
        codes[i] = to_e4m3(np.ldexp(X[i].astype(np.float64), e))
        scales[i] = np.float32(2.0 ** -e)
    return codes, scales
