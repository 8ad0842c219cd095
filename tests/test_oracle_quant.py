"""Pins for the format definitions used by the oracle (CPU only).

Expected codes follow from the bfloat16 and OCP FP8 E4M3 definitions by hand:
bf16 spacing at 1 is 2^-7, E4M3 spacing at 1 is 2^-3, E4M3 bias 7, max 448.
"""
import math

import numpy as np
import pytest

from oracle import quant as q


@pytest.mark.parametrize("x,bits", [
    (1.0, 0x3F80), (1 + 2 ** -8, 0x3F80), (1 + 3 * 2 ** -8, 0x3F82), (0.5, 0x3F00),
    (-2.0, 0xC000), (2 ** -126, 0x0080), (3.0, 0x4040), (1 + 2 ** -7, 0x3F81),
])
def test_bf16_codes(x, bits):
    assert q.bf16_bits(x) == bits


@pytest.mark.parametrize("x,bits", [
    (448.0, 0x7E), (2 ** -9, 0x01), (2 ** -6, 0x08), (1.0, 0x38), (0.1, 0x1D),
    (1 + 1 / 16, 0x38), (1 + 3 / 16, 0x3A), (460.0, 0x7E), (7 * 2 ** -9, 0x07),
    (2 ** -10, 0x00), (3 * 2 ** -10, 0x02), (240.0, 0x77),
])
def test_fp8_codes(x, bits):
    assert q.fp8_bits(x) == bits


def test_fp8_roundtrip_all_finite_codes():
    for b in range(0x7F):
        assert q.fp8_bits(q.fp8_from_bits(b)) == b


def test_error_bounds_random():
    rng = np.random.default_rng(0)
    for v in rng.random(3000) ** 4:
        c = float(v)
        assert abs(q.bf16_round(c) - c) <= 2 ** -8 * c
        r = q.fp8_round(c * 448)
        assert abs(r - c * 448) <= max(2 ** -4 * c * 448, 2 ** -10)


def test_fp8_scale():
    for cmax in (0.3, 1.0, 448.0, 448.1, 1e-5, 0.0017):
        e = q.fp8_scale_exp(cmax)
        assert cmax <= math.ldexp(448.0, e)
        assert cmax > math.ldexp(448.0, e - 1)
