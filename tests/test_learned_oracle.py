"""Pins of the learned-correction reference (CPU): BF16 rounding against exact
bit patterns, the analytic gradient against central differences, and the
zero-output start."""
import numpy as np
import pytest

from oracle import learned as LN


def test_bf16_rounding_bit_patterns():
    u = np.array([0x3F800000, 0x3F808000, 0x3F818000, 0x3F808001, 0xBF7FFFFF, 0x00000001], dtype=np.uint32)
    want = np.array([0x3F800000, 0x3F800000, 0x3F820000, 0x3F810000, 0xBF800000, 0x00000000], dtype=np.uint32)
    got = LN.bf16(u.view(np.float32)).view(np.uint32)
    assert np.array_equal(got, want)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    w = rng.normal(0, 0.4, LN.NPARAM)
    x = rng.normal(0, 1, (40, 32))
    g = rng.normal(0, 1, 40)
    c, cache = LN.forward(w, x, round_activations=False)
    grad = LN.backward(w, cache, g, round_weights=False)
    f = lambda ww: float(g @ LN.forward(ww, x, round_activations=False)[0])
    h = 1e-6
    idx = rng.choice(LN.NPARAM, 60, replace=False)
    idx = np.union1d(idx, [0, 511, 512, 527, 528, 783, 784, 799, 800, 815, 816])
    for p in idx:
        e = np.zeros(LN.NPARAM)
        e[p] = h
        fd = (f(w + e) - f(w - e)) / (2 * h)
        assert fd == pytest.approx(grad[p], rel=1e-6, abs=1e-7), p


def test_zero_output_layer_gives_zero_correction():
    w = LN.init_weights(0)
    x = np.random.default_rng(1).normal(0, 1, (10, 32)).astype(np.float32)
    c, _ = LN.forward(w, x)
    assert np.all(c == 0)
