"""Pins of the oracle's bfloat16 rounding and hi/lo split (CPU only).

The rounding is checked against torch's float32 -> bfloat16 conversion (an independent
library routine, round to nearest even), against hand-worked ties and boundaries, and
against the direct-rounding property for float64 inputs that rounding through float32
would break.
"""
import numpy as np
import pytest
import torch

from oracle import split


def _torch_bf16(x32: np.ndarray) -> np.ndarray:
    return torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()


def test_matches_torch_on_float32_inputs():
    rng = np.random.default_rng(7)
    parts = [
        rng.standard_normal(20000),
        rng.standard_normal(5000) * 1e-30,
        rng.standard_normal(5000) * 1e30,
        np.ldexp(rng.uniform(1, 2, 5000), rng.integers(-149, -126, 5000)),   # subnormal range
        np.ldexp(rng.uniform(1, 2, 2000), rng.integers(120, 128, 2000)),
    ]
    x32 = np.concatenate(parts).astype(np.float32)
    # exact ties: 8 significant bits plus a trailing one bit
    m = rng.integers(1 << 8, 1 << 9, 4000)
    ties = np.ldexp((2 * m + 1).astype(np.float64), rng.integers(-20, 20, 4000)).astype(np.float32)
    x32 = np.concatenate([x32, ties, -ties])
    got = split.round_bf16(x32.astype(np.float64))
    ref = _torch_bf16(x32)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("x,expect", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                                # tie, even neighbour is 1
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),                # tie, even neighbour is above
    (1.0 + 2.0 ** -8 + 2.0 ** -40, 1.0 + 2.0 ** -7),       # just above the tie (float64 only)
    (-(1.0 + 2.0 ** -8 + 2.0 ** -40), -(1.0 + 2.0 ** -7)),
    (3.0 * 2.0 ** -134, 2.0 ** -132),                      # subnormal tie 1.5 q -> 2 q
    (2.0 ** -134, 0.0),                                    # half the smallest subnormal -> 0 (even)
    (split.BF16_MAX, split.BF16_MAX),
    ((2.0 - 2.0 ** -8) * 2.0 ** 127 - 2.0 ** 100, split.BF16_MAX),
    ((2.0 - 2.0 ** -8) * 2.0 ** 127, np.inf),              # tie with the overflow boundary
    (0.0, 0.0),
    (np.inf, np.inf),
])
def test_hand_cases(x, expect):
    assert split.round_bf16(np.array([x]))[0] == expect


def test_float64_rounded_directly_not_through_float32():
    x = 1.0 + 2.0 ** -8 + 2.0 ** -40
    via32 = _torch_bf16(np.array([x], dtype=np.float32))[0]
    assert via32 == 1.0 and split.round_bf16(np.array([x]))[0] == 1.0 + 2.0 ** -7


def test_split_error_bounds_and_exact_cases():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(50000)
    hi, lo = split.split_hilo(x)
    assert np.array_equal(split.round_bf16(hi), hi) and np.array_equal(split.round_bf16(lo), lo)
    # unit roundoff of 8 significant bits is 2^-8: |x - hi| <= 2^-8 |x|, and the lo plane
    # leaves at most 2^-8 of that
    assert np.all(np.abs(x - hi) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))
    assert np.max(np.abs(x - hi - lo) / np.abs(x)) > 2.0 ** -18   # and the bound is not loose
    # numbers with at most 16 significant bits split exactly
    v = np.ldexp(rng.integers(1 << 15, 1 << 16, 1000).astype(np.float64), rng.integers(-30, 30, 1000))
    h2, l2 = split.split_hilo(v)
    assert np.array_equal(h2 + l2, v)


def test_bit_encoding():
    vals = np.array([1.0, -2.0, np.inf, 0.0, 2.0 ** -133, split.BF16_MAX])
    bits = split.bf16_bits(vals)
    assert list(bits) == [0x3F80, 0xC000, 0x7F80, 0x0000, 0x0001, 0x7F7F]
    assert np.array_equal(split.from_bf16_bits(bits), vals)
