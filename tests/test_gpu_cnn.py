"""Learned-direction network on the matrix cores against the FP64 oracle:
inference, loss and weight gradients (bf16 activations and weights, FP32
accumulation; relative L2 within 2e-2), the Adam update, the fixed point
d(0, m) = 0, sampled windows of a full-size image, the fused second and third
layers against separate ones (bitwise), and argument errors."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import cnn

pytestmark = pytest.mark.gpu

TOL = 2e-2


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def images(B, H, W, seed):
    """Seeded (g, m, s) images: smooth gradients, slowness-squared models and
    steps correlated with -g (the shape of optimiser steps)."""
    r = np.random.default_rng(seed)
    g = np.stack([synth.smooth(r.standard_normal((H, W)), 2.0) for _ in range(B)])
    g *= 1e-3 / np.abs(g).max()
    v = np.stack([2000.0 + 1500.0 * np.arange(H)[:, None] / H + synth.smooth(200 * r.standard_normal((H, W)), 3.0)
                  for _ in range(B)])
    m = 1.0 / v ** 2
    s = -(g + 0.5 * np.stack([synth.smooth(r.standard_normal((H, W)), 1.0) for _ in range(B)]) * 1e-3)
    return g.astype(np.float32), m.astype(np.float32), s.astype(np.float32)


def weights(seed, gate=10.0):
    ws = cnn.init_weights(np.random.default_rng(seed))
    ws[3] = ws[3] * gate  # spread z so that the gate is not constant
    return [cnn.bf16_round(w).reshape(w.shape) for w in ws]


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def case():
    B, H, W = 3, 37, 53  # 5883 pixels: ragged against 16-pixel MFMA tiles and 2048-pixel gradient chunks
    return weights(7), images(B, H, W, 11)


def test_forward_matches_oracle(case):
    from paper_2008_11778_amd import CNN
    ws, (g, m, s) = case
    B, H, W = g.shape
    with CNN(H, W, 4, ws) as net:
        z, d = net.forward(to_dev(g), to_dev(m))
        z, d = z.cpu().numpy(), d.cpu().numpy()
    for b in range(B):
        z_ref, d_ref = cnn.forward(ws, g[b], m[b])
        assert np.std(z_ref) > 0.1
        assert rel(z[b], z_ref) <= TOL, b
        assert rel(d[b], d_ref) <= TOL, b


def test_direction_fixed_point_and_descent(case):
    import torch
    from paper_2008_11778_amd import CNN
    ws, (g, m, _) = case
    B, H, W = g.shape
    with CNN(H, W, B, ws) as net:
        _, d0 = net.forward(torch.zeros(B, H, W, device="cuda"), to_dev(m))
        _, d = net.forward(to_dev(g), to_dev(m))
        assert torch.count_nonzero(d0).item() == 0
        for b in range(B):
            assert float((d[b].double() * to_dev(g)[b].double()).sum()) > 0.0


def test_gradients_match_oracle(case):
    from paper_2008_11778_amd import CNN
    from paper_2008_11778_amd._lib import cnn_unflatten
    ws, (g, m, s) = case
    B, H, W = g.shape
    with CNN(H, W, B, ws) as net:
        grad, loss = net.gradients(to_dev(g), to_dev(m), to_dev(s))
        grad, loss = grad.cpu().numpy(), float(loss.item())
    loss_ref, grads_ref = cnn.loss_and_grads(ws, list(zip(g, m, s)))
    assert abs(loss - loss_ref) <= TOL * loss_ref
    for li, (a, b) in enumerate(zip(cnn_unflatten(grad), grads_ref)):
        assert rel(a, b) <= TOL, (li, rel(a, b))


def test_adam_step_matches_closed_form(case):
    """First Adam step: w1 = w0 - lr * g / (|g| + eps) with the network's own
    gradient g (bias corrections cancel at step one)."""
    from paper_2008_11778_amd import CNN
    from paper_2008_11778_amd._lib import cnn_flatten
    ws, (g, m, s) = case
    B, H, W = g.shape
    lr = 1e-3
    with CNN(H, W, B, ws) as net:
        w0 = net.get_weights()
        assert np.array_equal(w0, cnn_flatten(ws))
        grad, _ = net.gradients(to_dev(g), to_dev(m), to_dev(s))
        gr = grad.cpu().numpy().astype(np.float64)
        net.train_step(to_dev(g), to_dev(m), to_dev(s), lr)
        w1 = net.get_weights()
    expect = w0 - lr * gr / (np.abs(gr) + 1e-8)
    np.testing.assert_allclose(w1, expect, rtol=0, atol=1e-6 * lr + 1e-7)


def test_training_lowers_the_loss(case):
    import torch
    from paper_2008_11778_amd import CNN
    ws, (g, m, s) = case
    B, H, W = g.shape
    with CNN(H, W, B, ws) as net:
        gd, md, sd = to_dev(g), to_dev(m), to_dev(s)
        losses = [float(net.train_step(gd, md, sd, 3e-3).item()) for _ in range(40)]
        torch.cuda.synchronize()
    # the FP64 oracle's Adam on the same batch goes 0.69 -> 0.42 in 40 steps
    assert losses[-1] < 0.75 * losses[0], (losses[0], losses[-1])
    loss_ref, _ = cnn.loss_and_grads(ws, list(zip(g, m, s)))
    assert abs(losses[0] - loss_ref) <= TOL * loss_ref


def test_full_size_sampled_windows():
    """A 384 x 1024 image batch (the learned-form model size), checked on
    windows: z at a pixel depends on the normalised inputs within 4 pixels,
    so the oracle's network on a window with a 4-pixel margin (clipped at the
    image edge, where zero padding applies in both) gives exact z there."""
    from paper_2008_11778_amd import CNN
    ws = weights(8)
    B, H, W = 2, 384, 1024
    g, m, _ = images(B, H, W, 12)
    with CNN(H, W, 8, ws) as net:
        z, _ = net.forward(to_dev(g), to_dev(m), d=False)
        z = z.cpu().numpy()
    r = np.random.default_rng(5)
    for b in range(B):
        x = cnn.normalise_inputs(g[b], m[b])
        for (y0, x0) in [(0, 0), (H - 16, W - 24), (int(r.integers(8, H - 24)), int(r.integers(8, W - 32)))]:
            y1, x1 = y0 + 16, x0 + 24
            ya, xa = max(y0 - 4, 0), max(x0 - 4, 0)
            yb, xb = min(y1 + 4, H), min(x1 + 4, W)
            h = x[:, ya:yb, xa:xb]
            for i, w in enumerate(ws):
                h = cnn.conv3x3(h, w)
                if i < 3:
                    h = np.maximum(h, 0.0)
            z_ref = h[0, y0 - ya:y1 - ya, x0 - xa:x1 - xa]
            assert rel(z[b, y0:y1, x0:x1], z_ref) <= TOL, (b, y0, x0)


@pytest.mark.parametrize("B,H,W", [(3, 37, 131), (2, 384, 1024)])
def test_fused_layers_bitwise(B, H, W):
    """Layers 2 and 3 in one kernel give bitwise the outputs of two separate
    kernels: the inference output z, and the weight gradient, which reads the
    second layer's activation that the fused training forward writes out.
    131 columns are two 62-column fused segments and a 7-column tail."""
    from paper_2008_11778_amd import CNN
    ws = weights(9)
    g, m, s = images(B, H, W, 13)
    out = {}
    with CNN(H, W, B, ws) as net:
        gd, md, sd = to_dev(g), to_dev(m), to_dev(s)
        for fused in (True, False):
            net.set_fused(fused)
            z, _ = net.forward(gd, md, d=False)
            grad, loss = net.gradients(gd, md, sd)
            out[fused] = (z.cpu().numpy(), grad.cpu().numpy(), float(loss.item()))
    assert np.std(out[True][0]) > 0.1
    assert np.array_equal(out[True][0], out[False][0])
    assert np.array_equal(out[True][1], out[False][1])
    assert out[True][2] == out[False][2]


def test_argument_errors(case):
    import torch
    from paper_2008_11778_amd import CNN
    from paper_2008_11778_amd._lib import _lib
    ws, (g, m, _) = case
    B, H, W = g.shape
    with CNN(H, W, 2, ws) as net:
        with pytest.raises(ValueError):
            net.forward(to_dev(g), to_dev(m))  # 3 images > max_batch 2
        gd, md = to_dev(g[:1]), to_dev(m[:1])
        out = torch.empty_like(gd)
        assert _lib.aafwi_cnn_forward(net._h, 0, gd.data_ptr(), md.data_ptr(), None, out.data_ptr()) == -1
        assert _lib.aafwi_cnn_forward(net._h, 3, gd.data_ptr(), md.data_ptr(), None, out.data_ptr()) == -1
        assert _lib.aafwi_cnn_train_step(net._h, 1, gd.data_ptr(), md.data_ptr(), gd.data_ptr(),
                                         ctypes.c_float(-1.0), None) == -1
    # one image above 2^25 pixels (its activations need 64-bit byte offsets) is refused before allocating
    from paper_2008_11778_amd._lib import cnn_flatten
    w = cnn_flatten(ws)
    h = ctypes.c_void_p()
    assert _lib.aafwi_cnn_create(8192, 4097, 1, w.ctypes.data, None, ctypes.byref(h)) == -1 and not h.value
