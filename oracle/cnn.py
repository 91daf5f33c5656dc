"""FP64 oracle of the learned upsampler (TEST INFRASTRUCTURE ONLY -- see
oracle/__init__).

The paper has no learned component; this is a stated reading of the upsampler
that reconstructs a full-resolution, fine-step render from a half-resolution,
coarse-step one:

  x   (H, W, 4) premultiplied RGBA of the coarse render
  a1 = relu(conv3x3(x;  W1 [32, 4, 3, 3],  b1[32]))
  a2 = relu(conv3x3(a1; W2 [32, 32, 3, 3], b2[32]))
  y  =      conv3x3(a2; W3 [16, 32, 3, 3], b3[16])
  out = pixel_shuffle2(y) + bilinear2(x)          (2H, 2W, 4), not clamped

conv3x3 is a cross-correlation with zero "same" padding:
  conv(x)[i, j, o] = b[o] + sum_{c, di, dj} W[o, c, di, dj] x[i + di - 1, j + dj - 1, c].
pixel_shuffle2 sends channel 4*c + 2*dy + dx of coarse pixel (i, j) to channel c
of fine pixel (2i + dy, 2j + dx).  bilinear2 samples the coarse image at fine
pixel centres mapped to coarse coordinates ((Y + 1/2)/2 - 1/2, (X + 1/2)/2 - 1/2)
with clamp-to-edge.  The loss is the mean squared error over all fine pixels and
the four channels; the optimiser is Adam (lr 1e-3, beta 0.9 / 0.999, eps 1e-8,
bias-corrected).

Precision reading of the device path: every layer's input (image or
activation) and its weights are rounded to bfloat16, products are accumulated
in FP32 with the bias, ReLU is applied and the result is rounded to bfloat16
for the next layer; the third layer's output, the pixel shuffle and the
bilinear residual stay FP32.  ``forward(..., bf16=True)`` applies the same
roundings (round to nearest even), and ``backward(..., bf16=True)`` those of
the backward pass (the output gradient and both hidden-layer gradients
rounded to bfloat16), so that the oracle and the device differ only by FP32
accumulation order.

Flat parameter layout (FP32 master copy): W1, b1, W2, b2, W3, b3, each
weight tensor [out][in][3][3] row-major.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((4, 32), (32, 32), (32, 16))
N_PARAMS = sum(co * ci * 9 + co for ci, co in LAYERS)


def split_params(p):
    """Flat vector -> [(W, b), ...] views."""
    p = np.asarray(p)
    out, off = [], 0
    for ci, co in LAYERS:
        w = p[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = p[off:off + co]
        off += co
        out.append((w, b))
    assert off == p.size
    return out


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 cin))), zero biases; the last layer is
    scaled by 0.1 so that the initial output is close to the bilinear image."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (ci, co) in enumerate(LAYERS):
        w = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci))
        if k == len(LAYERS) - 1:
            w *= 0.1
        parts += [w.reshape(-1), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as FP64 values."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u | 0x00400000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, w, b):
    """Cross-correlation with zero 'same' padding: x (H, W, Cin), w (Cout, Cin, 3, 3)."""
    H, W, _ = x.shape
    xp = np.zeros((H + 2, W + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    out = np.broadcast_to(np.asarray(b, np.float64), (H, W, w.shape[0])).copy()
    for di in range(3):
        for dj in range(3):
            out += xp[di:di + H, dj:dj + W] @ np.asarray(w[:, :, di, dj], np.float64).T
    return out


def conv3x3_backward(x, w, g):
    """Gradients of sum(g * conv3x3(x, w, b)) with respect to x, w and b."""
    H, W, _ = x.shape
    xp = np.zeros((H + 2, W + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    gx_p = np.zeros_like(xp)
    gw = np.zeros(w.shape)
    for di in range(3):
        for dj in range(3):
            wt = np.asarray(w[:, :, di, dj], np.float64)          # (Cout, Cin)
            gx_p[di:di + H, dj:dj + W] += g @ wt
            gw[:, :, di, dj] = np.einsum("hwo,hwc->oc", g, xp[di:di + H, dj:dj + W])
    return gx_p[1:-1, 1:-1], gw, g.sum(axis=(0, 1))


def pixel_shuffle2(y):
    """(H, W, 4C) -> (2H, 2W, C): channel 4c + 2dy + dx -> fine (2i+dy, 2j+dx, c)."""
    H, W, C4 = y.shape
    C = C4 // 4
    return y.reshape(H, W, C, 2, 2).transpose(0, 3, 1, 4, 2).reshape(2 * H, 2 * W, C)


def pixel_unshuffle2(z):
    """Inverse of pixel_shuffle2."""
    H2, W2, C = z.shape
    return z.reshape(H2 // 2, 2, W2 // 2, 2, C).transpose(0, 2, 4, 1, 3).reshape(H2 // 2, W2 // 2, 4 * C)


def _bilinear_taps(n):
    """Coarse taps and weights for fine coordinates 0..2n-1 (half-pixel centres,
    clamp to edge)."""
    c = (np.arange(2 * n) + 0.5) / 2.0 - 0.5
    i0 = np.floor(c).astype(np.int64)
    f = c - i0
    return np.clip(i0, 0, n - 1), np.clip(i0 + 1, 0, n - 1), f


def bilinear2(x):
    H, W, _ = x.shape
    y0, y1, fy = _bilinear_taps(H)
    x0, x1, fx = _bilinear_taps(W)
    fy = fy[:, None, None]
    fx = fx[None, :, None]
    top = x[y0][:, x0] * (1 - fx) + x[y0][:, x1] * fx
    bot = x[y1][:, x0] * (1 - fx) + x[y1][:, x1] * fx
    return top * (1 - fy) + bot * fy


def bilinear2_backward(x_shape, g):
    """Gradient of sum(g * bilinear2(x)) with respect to x."""
    H, W, C = x_shape
    y0, y1, fy = _bilinear_taps(H)
    x0, x1, fx = _bilinear_taps(W)
    gx = np.zeros((H, W, C))
    for Y in range(2 * H):
        for ya, wy in ((y0[Y], 1 - fy[Y]), (y1[Y], fy[Y])):
            row = g[Y] * wy                                   # (2W, C)
            np.add.at(gx[ya], x0, row * (1 - fx)[:, None])
            np.add.at(gx[ya], x1, row * fx[:, None])
    return gx


def forward(params, x, bf16=False):
    """Returns (out, cache).  x (H, W, 4)."""
    (w1, b1), (w2, b2), (w3, b3) = split_params(np.asarray(params, np.float64))
    q = bf16_round if bf16 else (lambda t: np.asarray(t, np.float64))
    x_in = q(x)
    w1q, w2q, w3q = q(w1), q(w2), q(w3)
    z1 = conv3x3(x_in, w1q, b1)
    a1 = q(np.maximum(z1, 0.0))
    z2 = conv3x3(a1, w2q, b2)
    a2 = q(np.maximum(z2, 0.0))
    y = conv3x3(a2, w3q, b3)
    out = pixel_shuffle2(y) + bilinear2(np.asarray(x, np.float64))
    cache = dict(x=x_in, w=(w1q, w2q, w3q), z1=z1, a1=a1, z2=z2, a2=a2)
    return out, cache


def loss(out, target):
    d = out - np.asarray(target, np.float64)
    return float(np.mean(d * d))


def backward(cache, out, target, bf16=False, count=None):
    """Gradient of the MSE loss with respect to the flat parameters (in the
    order of split_params).  The residual bilinear path has no parameters.

    ``count`` is the number of elements the mean runs over (default: this
    image's; a batch passes its total and sums the per-image results).
    ``bf16=True`` is the precision reading of the device's backward pass: the
    gradient of the last layer's output and the masked gradients of both hidden
    layers are rounded to bfloat16 (round to nearest even) before they enter
    the next convolution, the weight gradients and the bias sums; the weights
    and activations are the BF16-rounded ones of the forward cache.  The oracle
    and the device then differ only by FP32 accumulation order."""
    q = bf16_round if bf16 else (lambda t: t)
    n = out.size if count is None else count
    g = 2.0 * (out - np.asarray(target, np.float64)) / n
    gy = q(pixel_unshuffle2(g))
    w1, w2, w3 = cache["w"]
    ga2, gw3, gb3 = conv3x3_backward(cache["a2"], w3, gy)
    gz2 = q(ga2 * (cache["z2"] > 0))
    ga1, gw2, gb2 = conv3x3_backward(cache["a1"], w2, gz2)
    gz1 = q(ga1 * (cache["z1"] > 0))
    _, gw1, gb1 = conv3x3_backward(cache["x"], w1, gz1)
    return np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2, gw3.ravel(), gb3])


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t counts from 1).  Returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
