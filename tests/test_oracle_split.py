"""Pins of the split-precision oracle: the bf16 rounding against torch's
independent CPU float32 -> bfloat16 conversion (round to nearest even), the
representation bound |x - hi - lo| <= 2^-16 |x|, and the product bound
|A Y - (hi hi + hi lo + lo hi)| <= 3 * 2^-16 |A||Y|.  CPU only."""
import numpy as np
import torch

from oracle import split


def test_rounding_matches_torch_bfloat16():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(100000).astype(np.float32) * np.float32(3.7)
    # exact ties: low 16 bits 0x8000, both parities of the kept bit
    mant = rng.integers(0, 128, 2000).astype(np.uint32) << np.uint32(16)   # both parities of the kept bit
    expo = rng.integers(100, 150, 2000).astype(np.uint32) << np.uint32(23)
    ties = expo | mant | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32), np.array([0.0, -0.0, 1.0], np.float32)])
    ours = split.bf16_rne_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_representation_bound():
    rng = np.random.default_rng(1)
    x = rng.uniform(-10, 10, 200000).astype(np.float32)
    hi, lo = split.split(x)
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(x.astype(np.float64)))
    # x - hi is exact in float32
    assert np.array_equal((x - hi).astype(np.float64), x.astype(np.float64) - hi.astype(np.float64))


def test_product_bound_and_exact_case():
    rng = np.random.default_rng(2)
    A = rng.uniform(0, 1, (60, 300)).astype(np.float32)
    Y = rng.uniform(0, 1, (300, 20)).astype(np.float32)
    exact = A.astype(np.float64) @ Y.astype(np.float64)
    p3 = split.product3(A, Y)
    bound = 3 * 2.0 ** -16 * (np.abs(A).astype(np.float64) @ np.abs(Y).astype(np.float64))
    assert np.all(np.abs(p3 - exact) <= bound)
    # a single bf16 product would miss the bound by far: the correction matters
    ah, _ = split.split(A)
    yh, _ = split.split(Y)
    one = ah.astype(np.float64) @ yh.astype(np.float64)
    assert np.max(np.abs(one - exact) / bound) > 10
    # inputs that are already bf16: lo = 0 and the product is exact
    Ab = split.split(A)[0]
    Yb = split.split(Y)[0]
    np.testing.assert_array_equal(split.product3(Ab, Yb), Ab.astype(np.float64) @ Yb.astype(np.float64))


def test_rhs_orientations():
    rng = np.random.default_rng(3)
    A = rng.uniform(0, 1, (40, 30)).astype(np.float32)
    Ht = rng.uniform(0, 1, (30, 5)).astype(np.float32)
    W = rng.uniform(0, 1, (40, 5)).astype(np.float32)
    np.testing.assert_allclose(split.rhs_w(A, Ht), A.astype(np.float64) @ Ht, rtol=1e-4)
    np.testing.assert_allclose(split.rhs_h(A, W), A.T.astype(np.float64) @ W, rtol=1e-4)
