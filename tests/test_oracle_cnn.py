"""Pins of the FP64 surrogate-network oracle: closed forms of the layers,
central finite differences of the whole model, and Adam's first step."""
import numpy as np
import pytest

from oracle import cnn_oracle as co


def test_conv_delta_kernels_are_shifts():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 3))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 1, 1, c] = 1.0                      # centre tap: identity
    assert np.array_equal(co.conv3x3(x, w, np.zeros(3)), x)
    w = np.zeros((1, 3, 3, 3))
    w[0, 0, 0, 2] = 1.0                           # upper-left tap of channel 2
    y = co.conv3x3(x, w, np.zeros(1))[..., 0]
    expect = np.zeros((2, 5, 6))
    expect[:, 1:, 1:] = x[:, :-1, :-1, 2]         # y[i,j] = x[i-1,j-1], zero outside
    assert np.array_equal(y, expect)
    assert np.allclose(co.conv3x3(x, np.zeros((4, 3, 3, 3)), np.arange(4.0)), np.arange(4.0))


def test_pool_and_gap_of_constants_and_ramps():
    x = np.full((1, 4, 6, 2), 3.5)
    assert np.array_equal(co.pool2(x), np.full((1, 2, 3, 2), 3.5))
    assert np.array_equal(co.gap(x), np.full((1, 2), 3.5))
    r = np.arange(16.0).reshape(1, 4, 4, 1)
    assert co.pool2(r)[0, 0, 0, 0] == (0 + 1 + 4 + 5) / 4
    assert co.gap(r)[0, 0] == 7.5


def test_bf16_rounding():
    assert co.bf16_round(1.0) == 1.0
    assert co.bf16_round(1.0 + 2.0 ** -9) == 1.0            # below half an ulp (2^-7)
    assert co.bf16_round(1.0 + 3 * 2.0 ** -9) == 1.0 + 2.0 ** -7
    assert co.bf16_round(1.0 + 2.0 ** -8) == 1.0            # tie to even
    assert co.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7


def test_layout_counts():
    spec, n = co.layout([32, 64, 128, 128, 256], 256, 65)
    convs = 32 * 9 + 32 + 64 * 9 * 32 + 64 + 128 * 9 * 64 + 128 + 128 * 9 * 128 + 128 + 256 * 9 * 128 + 256
    assert n == convs + 256 * 256 + 256 + 65 * 256 + 65


@pytest.mark.parametrize("seed", [0, 1])
def test_model_gradient_matches_finite_differences(seed):
    m = co.Model([4, 4, 4, 4, 4], 6, 3)
    p = co.he_init(m.spec, m.n, seed) + 0.01
    rng = np.random.default_rng(seed + 10)
    imgs = (rng.random((2, 16, 16)) < 0.4).astype(np.uint8)
    tgt = rng.normal(size=(2, 3))
    y = m.forward(p, imgs)
    loss, dy = co.mse(y, tgt)
    g = m.backward(p, dy)
    idx = rng.choice(m.n, 60, replace=False)
    h = 1e-6
    for i in idx:
        pp = p.copy(); pp[i] += h
        lp = co.mse(m.forward(pp, imgs), tgt)[0]
        pm = p.copy(); pm[i] -= h
        lm = co.mse(m.forward(pm, imgs), tgt)[0]
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-4, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = co.adam(p, g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
