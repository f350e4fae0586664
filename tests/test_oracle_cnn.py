"""Pins for the CNN-preconditioner oracle: convolution against scipy's
correlate2d, hand-written backward against central differences, the fixed
point and descent properties of d_theta, Adam against its closed form for a
constant gradient, and bfloat16 rounding against known bit patterns."""
import numpy as np
from scipy.signal import correlate2d

from oracle import cnn


def test_conv3x3_matches_correlate2d():
    r = np.random.default_rng(0)
    x = r.standard_normal((3, 9, 11))
    w = r.standard_normal((4, 3, 3, 3))
    y = cnn.conv3x3(x, w)
    for co in range(4):
        ref = sum(correlate2d(x[ci], w[co, ci], mode="same", boundary="fill") for ci in range(3))
        np.testing.assert_allclose(y[co], ref, rtol=1e-12, atol=1e-12)


def test_conv_adjoints():
    r = np.random.default_rng(1)
    x = r.standard_normal((3, 8, 10))
    w = r.standard_normal((5, 3, 3, 3))
    dy = r.standard_normal((5, 8, 10))
    lhs = float(np.sum(cnn.conv3x3(x, w) * dy))
    assert abs(lhs - float(np.sum(x * cnn.conv3x3_input_grad(dy, w)))) < 1e-10 * abs(lhs)
    assert abs(lhs - float(np.sum(w * cnn.conv3x3_weight_grad(dy, x)))) < 1e-10 * abs(lhs)


def _tiny_batch(seed=2, B=2, H=10, W=12):
    r = np.random.default_rng(seed)
    out = []
    for _ in range(B):
        g = r.standard_normal((H, W))
        m = 1.0 + 0.1 * r.standard_normal((H, W))
        s = -(g + 0.3 * r.standard_normal((H, W)))
        out.append((g, m, s))
    return out


def test_backward_matches_central_differences():
    r = np.random.default_rng(3)
    ws = cnn.init_weights(r)
    ws[3] *= 10.0  # make the gate non-trivial
    batch = _tiny_batch()
    loss, grads = cnn.loss_and_grads(ws, batch)
    for li in range(4):
        dw = r.standard_normal(ws[li].shape)
        eps = 1e-6
        wp = [w.copy() for w in ws]
        wm = [w.copy() for w in ws]
        wp[li] += eps * dw
        wm[li] -= eps * dw
        fd = (cnn.loss_and_grads(wp, batch)[0] - cnn.loss_and_grads(wm, batch)[0]) / (2 * eps)
        an = float(np.sum(grads[li] * dw))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-8), (li, fd, an)


def test_direction_keeps_fixed_point_and_descends():
    r = np.random.default_rng(4)
    ws = cnn.init_weights(r)
    m = 1.0 + 0.1 * r.standard_normal((8, 8))
    z, d = cnn.forward(ws, np.zeros((8, 8)), m)
    assert np.all(d == 0.0)
    g = r.standard_normal((8, 8))
    z, d = cnn.forward(ws, g, m)
    assert float(np.sum(d * g)) > 0.0


def test_loss_is_zero_for_a_perfect_prediction_and_scale_free():
    r = np.random.default_rng(5)
    g = r.standard_normal((6, 7))
    z = r.standard_normal((6, 7))
    d = cnn.softplus(z) * g
    loss, dz = cnn.loss_and_dz(z, g, d / np.sqrt(np.mean(d * d)))
    assert loss < 1e-28 and np.abs(dz).max() < 1e-12
    s = r.standard_normal((6, 7))
    a = cnn.loss_and_dz(z, g, cnn.target(s))[0]
    b = cnn.loss_and_dz(z, 7.0 * g, cnn.target(3.0 * s))[0]
    assert abs(a - b) < 1e-12


def test_adam_closed_form_for_constant_gradient():
    ws = [np.zeros(3)]
    opt = cnn.Adam(ws, lr=0.1)
    g = [np.array([1.0, -2.0, 0.5])]
    for _ in range(5):
        ws = opt.step(ws, g)
    # with a constant gradient the bias-corrected ratio is sign(g) up to eps
    np.testing.assert_allclose(ws[0], -0.5 * np.sign(g[0]), rtol=1e-6)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, 3.14159265, -2.5e-3], np.float32)
    y = cnn.bf16_round(x)
    assert y[0] == 1.0
    assert y[1] == 1.0                 # halfway, ties to even
    assert y[2] == 1.0078125           # above halfway rounds up
    assert abs(y[3] - 3.140625) < 1e-12
    assert abs(y[4] - (-0.0025024414)) < 1e-9
