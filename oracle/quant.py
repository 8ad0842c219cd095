"""Reduced-precision formats, from their definitions — TEST INFRASTRUCTURE ONLY.

  * bfloat16: binary32's sign and 8-bit exponent with an 8-bit significand
    (7 stored bits); rounding to nearest, ties to even.
  * FP8 E4M3 (OCP 8-bit floating point, E4M3 encoding): exponent bias 7,
    3 stored mantissa bits, largest finite value 448, smallest normal 2^-6,
    subnormal spacing 2^-9, no infinities; here with saturation at 448.
  * Per-centroid FP8 scale: the power of two sigma = 2^e with e the least
    integer such that max_t c_t <= 448 * 2^e, so scaling is exact.

Rounding is done exactly: the spacing (ulp) at the value's binade is a power of
two, so value / ulp is exact in double and Python's round() rounds half to even.
"""
from __future__ import annotations

import math
import struct

import numpy as np


def _rne_to_grid(v: float, ulp: float) -> float:
    return round(v / ulp) * ulp   # round(): half to even, exact here


def bf16_round(c: float) -> float:
    """Nearest bfloat16 value (ties to even) of a double."""
    if c == 0.0 or not math.isfinite(c):
        return c
    m, e = math.frexp(abs(c))          # |c| = m * 2^e, 0.5 <= m < 1
    ulp = max(math.ldexp(1.0, e - 8), math.ldexp(1.0, -133))
    q = _rne_to_grid(abs(c), ulp)
    if q > 3.3895313892515355e38:       # beyond the largest finite bfloat16
        q = math.inf
    return math.copysign(q, c)


def bf16_bits(c: float) -> int:
    q = bf16_round(c)
    return struct.unpack("<I", struct.pack("<f", q))[0] >> 16


def bf16_from_bits(b: int) -> float:
    return struct.unpack("<f", struct.pack("<I", (int(b) & 0xFFFF) << 16))[0]


FP8_MAX = 448.0


def fp8_round(v: float) -> float:
    """Nearest E4M3 value (ties to even, saturating at 448) of a non-negative
    double."""
    if v < 0 or not math.isfinite(v):
        raise ValueError("non-negative finite values only")
    if v == 0.0:
        return 0.0
    m, e = math.frexp(v)               # v in [2^(e-1), 2^e)
    ulp = max(math.ldexp(1.0, e - 4), math.ldexp(1.0, -9))
    q = _rne_to_grid(v, ulp)
    return min(q, FP8_MAX)


def fp8_bits(v: float) -> int:
    q = fp8_round(v)
    if q == 0.0:
        return 0
    if q >= math.ldexp(1.0, -6):
        m, e = math.frexp(q)           # q = m * 2^e, m in [0.5, 1)
        E = e - 1 + 7                  # biased exponent
        M = int(round((m * 2 - 1) * 8))
        return (E << 3) | M
    return int(round(q / math.ldexp(1.0, -9)))


def fp8_from_bits(b: int) -> float:
    b = int(b) & 0xFF
    s = -1.0 if b & 0x80 else 1.0
    E = (b >> 3) & 0xF
    M = b & 0x7
    if E == 0xF and M == 0x7:
        return math.nan
    if E == 0:
        return s * M * math.ldexp(1.0, -9)
    return s * (1 + M / 8.0) * math.ldexp(1.0, E - 7)


def fp8_scale_exp(cmax: float) -> int:
    """Least e with cmax <= 448 * 2^e (0 when cmax == 0)."""
    if cmax <= 0.0:
        return 0
    _, e = math.frexp(cmax / FP8_MAX)
    e += 1
    while e > -1074 and cmax <= math.ldexp(FP8_MAX, e - 1):
        e -= 1
    while cmax > math.ldexp(FP8_MAX, e):
        e += 1
    return e


def quantize_row(row: np.ndarray, precision: str):
    """Scoring copy of one centroid: (codes, scale).  codes are uint32 float
    bits (fp32), uint16 (bf16) or uint8 (fp8); scale is 2^e (fp8) or 1."""
    if precision == "fp32":
        return row.astype(np.float32).view(np.uint32), 1.0
    if precision == "bf16":
        return np.array([bf16_bits(float(c)) for c in row], dtype=np.uint16), 1.0
    if precision == "fp8":
        e = fp8_scale_exp(float(np.max(row)) if row.size else 0.0)
        return (np.array([fp8_bits(math.ldexp(float(c), -e)) for c in row], dtype=np.uint8),
                math.ldexp(1.0, e))
    raise ValueError(precision)
