"""Pins of the oracle's reduced-precision quantizers against library
conversions that implement the same IEEE rounding (round to nearest even)."""
import numpy as np
import pytest
import torch

import oracle


def _edge_f32():
    rng = np.random.default_rng(0)
    vals = [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.99, 65520.0, 1e6, -1e6,
            2.0 ** -14, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -26, 1e-10,
            1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8,
            np.inf, -np.inf, 3.4e38, 1.1754944e-38, 1e-45]
    r = np.concatenate([np.array(vals), rng.standard_normal(4000) * 10.0 ** rng.uniform(-9, 6, 4000)])
    return r.astype(np.float32)


def test_f16_matches_ieee_conversion():
    x = _edge_f32()
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    got = np.array([oracle.f32_to_f16_bits(float(v)) for v in x], dtype=np.uint16)
    np.testing.assert_array_equal(got, ref)


def test_bf16_matches_torch_conversion():
    x = _edge_f32()
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = np.array([oracle.f32_to_bf16_bits(float(v)) for v in x], dtype=np.uint16)
    np.testing.assert_array_equal(got, ref)


def test_bulk_quantizers_are_elementwise():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000) * 3.0
    np.testing.assert_array_equal(
        oracle.bf16_bits(x), [oracle.f32_to_bf16_bits(float(np.float32(v))) for v in x])
    e = oracle.f16_block_exponent(x)
    np.testing.assert_array_equal(
        oracle.f16_scaled_bits(x, e),
        (x * 2.0 ** e).astype(np.float32).astype(np.float16).view(np.uint16))


@pytest.mark.parametrize("scale", [1e-20, 1e-6, 1.0, 3.0, 7e4, 1e20])
def test_f16_block_exponent_range(scale):
    x = np.random.default_rng(1).standard_normal(500) * scale
    e = oracle.f16_block_exponent(x)
    amax = np.abs(x).max() * 2.0 ** e
    assert 2.0 ** 13 <= amax < 2.0 ** 14
    assert oracle.f16_block_exponent(np.zeros(4)) == 0
