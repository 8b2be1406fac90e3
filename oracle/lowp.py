"""Rounding to the low-precision storage formats of the precision form (test
infrastructure only).

The paper analyses the method in one working precision (Theorem 3 bounds the error
of the indicator by the unit roundoff u); its precision form here stores A and the
sketch operands in bfloat16 and lets everything the error indicator depends on run
in binary64.  These functions define the roundings on binary64 values directly from
the mathematics of the formats, independent of any library conversion:

* bfloat16: 1 sign bit, 8 exponent bits (bias 127, the exponent range of binary32),
  7 stored significand bits; normal numbers carry 8 significant bits, subnormals a
  fixed quantum of 2^-133; values beyond the largest finite number
  (2 - 2^-7) 2^127 round to infinity as in IEEE 754 round-to-nearest.
* OCP e4m3fn (the 8-bit format with 4 exponent bits, bias 7, and 3 stored significand
  bits, without infinities): normal numbers 2^(e-7) (1 + m/8) for e = 1..15 carry 4
  significant bits, except that e = 15, m = 7 encodes NaN, so the largest finite value is
  1.75 * 2^8 = 448; subnormals m 2^-9 for m = 1..7.  A value whose rounding would exceed
  448 has no e4m3 representation (NaN here).
* round to nearest, ties to even, applied once to the binary64 value (no rounding
  through binary32 first, which could round twice).
"""
from __future__ import annotations

import numpy as np

BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127
BF16_MIN_NORMAL = 2.0 ** -126
BF16_QUANTUM_SUB = 2.0 ** -133


def round_bf16(x) -> np.ndarray:
    """Round binary64 values to the nearest bfloat16 value (ties to even); the result
    is returned as binary64 holding the bfloat16 value exactly."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    ax = np.abs(x)
    finite = np.isfinite(x)
    # normal range: 8 significant bits.  frexp gives x = f 2^e with 1/2 <= |f| < 1, so
    # the bfloat16 neighbours are multiples of 2^(e - 8).
    f, e = np.frexp(np.where(finite, x, 0.0))
    normal = finite & (ax >= BF16_MIN_NORMAL)
    q = np.rint(f * 256.0)                       # rint rounds half to even
    out_normal = np.ldexp(q, e - 8)
    # subnormal range: multiples of 2^-133
    out_sub = np.rint(x * 2.0 ** 133) * BF16_QUANTUM_SUB
    out = np.where(normal, out_normal, out_sub)
    # overflow: a value at or beyond the midpoint between the largest finite number
    # and 2^128 rounds to infinity (the midpoint itself is a tie whose even neighbour
    # is 2^128)
    over = finite & (np.abs(out) > BF16_MAX)
    out = np.where(over, np.copysign(np.inf, x), out)
    out = np.where(finite, out, x)
    # keep the sign of zero
    out = np.where(out == 0.0, np.copysign(0.0, x), out)
    return out


def is_bf16(x) -> bool:
    """True when every entry of x is a bfloat16 value."""
    x = np.asarray(x, dtype=np.float64)
    return bool(np.array_equal(round_bf16(x), x, equal_nan=True))


E4M3_MAX = 448.0
E4M3_MIN_NORMAL = 2.0 ** -6
E4M3_QUANTUM_SUB = 2.0 ** -9


def round_e4m3(x) -> np.ndarray:
    """Round binary64 values to the nearest OCP e4m3fn value (ties to even); the result is
    returned as binary64 holding the e4m3 value exactly.  Values that would round beyond
    448 (and NaN inputs) give NaN; the format has no infinity."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    finite = np.isfinite(x)
    # normal range: 4 significant bits; frexp gives x = f 2^e with 1/2 <= |f| < 1, so the
    # e4m3 neighbours are multiples of 2^(e - 4)
    f, e = np.frexp(np.where(finite, x, 0.0))
    normal = finite & (ax >= E4M3_MIN_NORMAL)
    out_normal = np.ldexp(np.rint(f * 16.0), e - 4)
    # subnormal range: multiples of 2^-9
    out_sub = np.rint(x * 2.0 ** 9) * E4M3_QUANTUM_SUB
    out = np.where(normal, out_normal, out_sub)
    out = np.where(finite & (np.abs(out) <= E4M3_MAX), out, np.nan)
    out = np.where(out == 0.0, np.copysign(0.0, x), out)
    return out


def is_e4m3(x) -> bool:
    """True when every entry of x is an e4m3fn value."""
    x = np.asarray(x, dtype=np.float64)
    return bool(np.array_equal(round_e4m3(x), x, equal_nan=True))
