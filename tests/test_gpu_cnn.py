"""The learned upsampler's HIP kernels (BF16 MFMA) against the FP64 oracle run
on the same BF16-rounded operands: inference, gradients, the Adam update and
bit-identical resume from a checkpoint.

Tolerances follow from the arithmetic: inference differs from the oracle only
by FP32 accumulation order (and the rare BF16 rounding flip of an activation
that this causes), so the relative Frobenius error is held to 1e-3; the
backward pass also rounds the output gradient and the hidden-layer gradients
to BF16, and the oracle's backward applies the same roundings, so gradients
are held to 1e-3 per parameter block as well."""
import numpy as np
import pytest

from oracle import cnn
from paper_1205_0282_amd import binding

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _images(rng, n, h, w):
    x = rng.uniform(0.0, 1.0, (n, h, w, 4)).astype(np.float32)
    x[..., :3] *= x[..., 3:4]                      # premultiplied
    x[:, : h // 3] *= 0.0                          # some transparent background
    t = rng.uniform(0.0, 1.0, (n, 2 * h, 2 * w, 4)).astype(np.float32)
    return x, t


@pytest.fixture(scope="module")
def caster():
    bc = binding.BrickCaster(0)
    bc.cnn_setup(2, 40, 52)
    yield bc
    bc.close()


def _params(seed):
    rng = np.random.default_rng(seed)
    p = cnn.init_params(seed)
    p[cnn.N_PARAMS - 16:] = rng.standard_normal(16).astype(np.float32) * 0.05
    p[1152:1184] = rng.standard_normal(32).astype(np.float32) * 0.05
    return p


@pytest.mark.parametrize("shape", [(1, 16, 16), (2, 37, 45), (1, 40, 52)])
def test_inference_matches_oracle(caster, shape):
    import torch
    n, h, w = shape
    rng = np.random.default_rng(h * w)
    p = _params(3)
    caster.cnn_set_weights(p)
    x, _ = _images(rng, n, h, w)
    out = caster.cnn_forward(torch.from_numpy(x).cuda()).cpu().numpy()
    for i in range(n):
        ref, _ = cnn.forward(p.astype(np.float64), x[i], bf16=True)
        assert _rel(out[i], ref) <= 1e-3, _rel(out[i], ref)
        assert np.abs(out[i] - ref).max() <= 2e-2


def test_zero_last_layer_is_exact_bilinear(caster):
    import torch
    p = _params(4)
    p[cnn.N_PARAMS - (16 * 32 * 9 + 16):] = 0.0
    caster.cnn_set_weights(p)
    x, _ = _images(np.random.default_rng(5), 1, 21, 30)
    out = caster.cnn_forward(torch.from_numpy(x).cuda()).cpu().numpy()[0]
    assert np.abs(out - cnn.bilinear2(x[0].astype(np.float64))).max() <= 1e-6


def test_gradients_match_oracle(caster):
    import torch
    n, h, w = 2, 24, 29
    rng = np.random.default_rng(6)
    p = _params(7)
    caster.cnn_set_weights(p)
    x, t = _images(rng, n, h, w)
    g_gpu, loss_gpu = caster.cnn_gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g_ref = np.zeros(cnn.N_PARAMS)
    loss_ref = 0.0
    for i in range(n):
        out, cache = cnn.forward(p.astype(np.float64), x[i], bf16=True)
        g_ref += cnn.backward(cache, out, t[i], bf16=True, count=n * out.size)
        loss_ref += cnn.loss(out, t[i]) / n
    assert abs(loss_gpu - loss_ref) <= 1e-3 * loss_ref
    blocks = [(0, 1152), (1152, 1184), (1184, 10400), (10400, 10432), (10432, 15040), (15040, 15056)]
    for lo, hi in blocks:
        rel = _rel(g_gpu[lo:hi], g_ref[lo:hi])
        print(f"parameters {lo}..{hi}: relative Frobenius error {rel:.3g}")
        assert rel <= 1e-3, (lo, hi, rel)


def test_adam_step_and_resume_bit_identical(caster):
    import torch
    n, h, w = 1, 32, 40
    rng = np.random.default_rng(8)
    x, t = _images(rng, n, h, w)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    p = _params(9)
    caster.cnn_set_weights(p)
    g, _ = caster.cnn_gradients(xd, td)
    caster.cnn_train_step(xd, td, lr=1e-3)
    w1, m1, v1, s1 = caster.cnn_get_weights()
    assert s1 == 1
    ref_p, ref_m, ref_v = cnn.adam_step(p.astype(np.float64), g.astype(np.float64), np.zeros(cnn.N_PARAMS),
                                        np.zeros(cnn.N_PARAMS), 1, lr=1e-3)
    assert np.abs(w1 - ref_p).max() <= 1e-6
    assert np.allclose(m1, ref_m, rtol=1e-6, atol=1e-12)
    # three more steps, checkpoint after the first of them
    losses = [caster.cnn_train_step(xd, td, lr=1e-3)]
    ck = caster.cnn_get_weights()
    losses += [caster.cnn_train_step(xd, td, lr=1e-3) for _ in range(2)]
    end = caster.cnn_get_weights()
    caster.cnn_set_weights(ck[0], ck[1], ck[2], ck[3])
    for _ in range(2):
        caster.cnn_train_step(xd, td, lr=1e-3)
    again = caster.cnn_get_weights()
    for a, b in zip(end[:3], again[:3]):
        assert np.array_equal(a, b)
    assert end[3] == again[3] == 4


def test_training_reduces_loss(caster):
    import torch
    n, h, w = 2, 32, 40
    rng = np.random.default_rng(10)
    x = rng.uniform(0, 1, (n, h, w, 4)).astype(np.float32)
    # target: a sharpened upsampling the network can learn
    t = np.stack([cnn.bilinear2(xi.astype(np.float64)) for xi in x])
    t = np.clip(t + 0.3 * (t - t.mean(axis=(1, 2), keepdims=True)), 0, 1).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    caster.cnn_set_weights(_params(11))
    first = caster.cnn_train_step(xd, td, lr=2e-3)
    for _ in range(60):
        last = caster.cnn_train_step(xd, td, lr=2e-3)
    assert last < 0.7 * first, (first, last)
