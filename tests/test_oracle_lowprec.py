"""Pins of the oracle's 16-bit value rounding against torch's CPU conversions
(an independent implementation of the same IEEE/bfloat16 rounding rule)."""

import numpy as np
import torch

from oracle import round_to_bf16, round_to_f16


def _samples():
    rng = np.random.default_rng(20)
    x = np.concatenate([rng.uniform(0, 1, 5000), rng.standard_normal(5000) * 1e-3,
                        np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.0, 2.0 ** -130])])
    return x.astype(np.float32).astype(np.float64)


def test_bf16_matches_torch():
    x = _samples()
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_to_bf16(x), ref)


def test_bf16_ties_to_even():
    assert round_to_bf16(1.0 + 2.0 ** -8) == 1.0                  # tie, even neighbour is 1.0
    assert round_to_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie, rounds up to even


def test_f16_matches_torch():
    x = _samples()
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_to_f16(x), ref)
