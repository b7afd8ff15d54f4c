"""Split-precision encoding of the design matrix for the BF16 precision form.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper computes in one precision throughout. The precision form stores X as two
bfloat16 planes, X = hi + lo with hi = bf16(X) and lo = bf16(X - hi), and forms each
product of X with an FP32 operand A = A_hi + A_lo as hi*A_hi + hi*A_lo + lo*A_hi (the
three-term "bf16x3" product of Henry, Tang and Heinecke, 2019). This module holds the
plain definitions that the device's encoding must reproduce bit for bit:

  * bfloat16 is a binary floating-point format with 8 significant bits (7 stored) and the
    exponent range of binary32: normal numbers down to 2^-126, subnormals spaced 2^-133,
    largest finite (2 - 2^-7) * 2^127;
  * bf16(x) rounds the exact value x to the nearest such number, ties to the one with an
    even last significant bit, and to +-inf beyond the largest finite value's rounding
    range. It is applied to the exact value (an FP64 input is rounded once, not through
    binary32 first).
"""
from __future__ import annotations

import numpy as np

BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127
_EMIN_NORMAL = -126          # smallest normal exponent: 2^-126
_SUB_QUANTUM = 2.0 ** -133   # spacing of the subnormals (2^-126 / 2^7)


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value of each element of float64 array x, as float64.

    For a nonzero normal result with 2^(e-1) <= |x| < 2^e, the representable neighbours
    are multiples of 2^(e-8) (8 significant bits); below 2^-126 they are multiples of
    2^-133. Dividing by that power of two is exact, numpy's rint rounds half to even, and
    multiplying back is exact, so the result is the correctly rounded value.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    fin = np.isfinite(x) & (x != 0.0)
    xf = x[fin]
    _, e = np.frexp(xf)                           # xf = f * 2^e, 0.5 <= |f| < 1
    q = np.where(e - 1 >= _EMIN_NORMAL, np.ldexp(1.0, e - 8), _SUB_QUANTUM)
    r = np.rint(xf / q) * q
    r = np.where(np.abs(r) > BF16_MAX, np.copysign(np.inf, r), r)
    out[fin] = r
    return out


def split_hilo(x) -> tuple[np.ndarray, np.ndarray]:
    """(hi, lo) with hi = bf16(x) and lo = bf16(x - hi), both float64 arrays of bf16 values.

    x - hi is formed exactly in float64 for float32 or bfloat16-representable inputs, and for
    float64 inputs whose rounding error is representable (all finite normal inputs of
    moderate exponent, which covers every workload here).
    """
    x = np.asarray(x, dtype=np.float64)
    hi = round_bf16(x)
    lo = round_bf16(x - hi)
    return hi, lo


def bf16_bits(v) -> np.ndarray:
    """The 16-bit encoding of bfloat16 values given as float64 (the upper half of binary32)."""
    v = np.asarray(v, dtype=np.float64)
    return (v.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    """float64 values of 16-bit bfloat16 encodings."""
    b = np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)
