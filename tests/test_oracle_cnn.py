"""Pins for the FP64 oracle of the learned upsampler: an independent library
correlation, finite differences, identities of the pixel shuffle and the
bilinear upsampler, closed forms of bf16 rounding and of the first Adam step."""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn


def _rng(s=0):
    return np.random.default_rng(s)


def test_conv_matches_scipy_correlate():
    rng = _rng(1)
    x = rng.standard_normal((9, 11, 3))
    w = rng.standard_normal((5, 3, 3, 3))
    b = rng.standard_normal(5)
    y = cnn.conv3x3(x, w, b)
    for o in range(5):
        ref = b[o] + sum(signal.correlate2d(x[:, :, c], w[o, c], mode="same", boundary="fill")
                         for c in range(3))
        assert np.allclose(y[:, :, o], ref, atol=1e-12)


def test_delta_kernel_is_identity_and_shift():
    rng = _rng(2)
    x = rng.standard_normal((6, 7, 4))
    w = np.zeros((4, 4, 3, 3))
    for c in range(4):
        w[c, c, 1, 1] = 1.0
    assert np.array_equal(cnn.conv3x3(x, w, np.zeros(4)), x)
    # tap (0, 1) reads the row above (zero padding at the top)
    w2 = np.zeros((1, 4, 3, 3))
    w2[0, 2, 0, 1] = 1.0
    y = cnn.conv3x3(x, w2, np.zeros(1))[:, :, 0]
    assert np.array_equal(y[1:], x[:-1, :, 2]) and np.all(y[0] == 0)


def test_pixel_shuffle_layout_and_inverse():
    y = np.arange(2 * 3 * 8, dtype=np.float64).reshape(2, 3, 8)
    z = cnn.pixel_shuffle2(y)
    assert z.shape == (4, 6, 2)
    for i in range(2):
        for j in range(3):
            for c in range(2):
                for dy in range(2):
                    for dx in range(2):
                        assert z[2 * i + dy, 2 * j + dx, c] == y[i, j, 4 * c + 2 * dy + dx]
    assert np.array_equal(cnn.pixel_unshuffle2(z), y)


def test_bilinear_exact_on_linear_ramp_and_constant():
    H, W = 7, 9
    i, j = np.mgrid[0:H, 0:W]
    x = np.stack([3.0 + 0.5 * i - 0.25 * j, np.full((H, W), 2.0)], axis=-1)
    up = cnn.bilinear2(x)
    Y, X = np.mgrid[0:2 * H, 0:2 * W]
    ci, cj = (Y + 0.5) / 2 - 0.5, (X + 0.5) / 2 - 0.5
    inner = (ci >= 0) & (ci <= H - 1) & (cj >= 0) & (cj <= W - 1)
    assert np.allclose(up[..., 0][inner], (3.0 + 0.5 * ci - 0.25 * cj)[inner], atol=1e-12)
    assert np.allclose(up[..., 1], 2.0, atol=1e-15)


def test_bilinear_backward_is_adjoint():
    rng = _rng(3)
    x = rng.standard_normal((5, 6, 2))
    g = rng.standard_normal((10, 12, 2))
    lhs = np.sum(g * cnn.bilinear2(x))
    rhs = np.sum(x * cnn.bilinear2_backward(x.shape, g))
    assert abs(lhs - rhs) < 1e-10


def test_gradients_match_central_differences():
    rng = _rng(4)
    p = cnn.init_params(5).astype(np.float64)
    p[cnn.N_PARAMS - 16:] = rng.standard_normal(16) * 0.1       # non-zero last biases
    x = rng.uniform(0, 1, (5, 6, 4))
    t = rng.uniform(0, 1, (10, 12, 4))
    out, cache = cnn.forward(p, x)
    g = cnn.backward(cache, out, t)
    h = 1e-6
    idx = np.concatenate([rng.choice(cnn.N_PARAMS, 60, replace=False), [0, 1152, 1184, 10400, 10432]])
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (cnn.loss(cnn.forward(pp, x)[0], t) - cnn.loss(cnn.forward(pm, x)[0], t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_bf16_rounding_closed_forms():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e38], np.float64)
    r = cnn.bf16_round(vals)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert r[3] == 1.0 + 2 ** -6
    assert r[4] == -2.5 and r[5] == 0.0
    rng = _rng(6)
    x = rng.standard_normal(10000) * 100
    q = cnn.bf16_round(x)
    assert np.all(np.abs(q - x.astype(np.float32)) <= np.abs(x) * 2 ** -8)
    assert np.array_equal(cnn.bf16_round(q), q)


def test_adam_first_step_closed_form():
    rng = _rng(7)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = cnn.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_zero_last_layer_gives_bilinear_output():
    p = cnn.init_params(8).astype(np.float64)
    off = cnn.N_PARAMS - (16 * 32 * 9 + 16)
    p[off:] = 0.0
    x = _rng(9).uniform(0, 1, (4, 5, 4))
    out, _ = cnn.forward(p, x)
    assert np.allclose(out, cnn.bilinear2(x), atol=1e-15)


def test_bf16_backward_is_the_exact_gradient_up_to_bf16_steps():
    """The BF16 reading of the backward pass stays within the rounding it
    models (relative step 2^-8 per rounded operand, three in series at the
    first layer) of the exact gradient of the same forward pass, and does round
    (it is not the exact gradient)."""
    rng = _rng(21)
    p = cnn.init_params(22).astype(np.float64)
    p[cnn.N_PARAMS - 16:] = rng.standard_normal(16) * 0.1
    x = rng.uniform(0, 1, (7, 9, 4))
    t = rng.uniform(0, 1, (14, 18, 4))
    out, cache = cnn.forward(p, x, bf16=True)
    g64 = cnn.backward(cache, out, t)
    g16 = cnn.backward(cache, out, t, bf16=True)
    blocks = [(0, 1152), (1152, 1184), (1184, 10400), (10400, 10432), (10432, 15040), (15040, 15056)]
    for lo, hi in blocks:
        rel = np.linalg.norm(g16[lo:hi] - g64[lo:hi]) / np.linalg.norm(g64[lo:hi])
        assert 0.0 < rel <= 3 * 2.0 ** -8, (lo, hi, rel)


def test_bf16_backward_last_layer_exact_when_output_gradient_is_representable():
    """With an output gradient whose every element is a power of two (exact in
    bfloat16) the last layer's weight and bias gradients of the BF16 reading
    equal the exact ones (to FP64 rounding): nothing else is rounded before
    them, while the earlier layers' gradients are rounded."""
    rng = _rng(23)
    p = cnn.init_params(24).astype(np.float64)
    x = rng.uniform(0, 1, (5, 6, 4))
    out, cache = cnn.forward(p, x, bf16=True)
    n = out.size
    step = 2.0 ** rng.integers(-6, 0, out.shape) * rng.choice([-1.0, 1.0], out.shape)
    t = out - step * n / 2.0          # 2 (out - t) / n = step, up to one FP64 rounding
    g64 = cnn.backward(cache, out, t)
    g16 = cnn.backward(cache, out, t, bf16=True)
    assert np.allclose(g16[10432:], g64[10432:], rtol=1e-12, atol=0.0)
    assert not np.array_equal(g16[:10432], g64[:10432])
