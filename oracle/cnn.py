"""FP64 oracle for the learned preconditioner of the Anderson step.
TEST INFRASTRUCTURE ONLY.

The network is not from the paper; it is the learned variant of the fixed
point map of Section "Method": G_theta(p) = p - eta d_theta(p) with
d_theta = softplus(z) * g, z = CNN([g_hat, m_hat]), so that d_theta = 0 exactly
when g = 0 (the fixed points of G in eq. GD are kept) and <d_theta, g> > 0
(a descent direction).  Inputs are scale-free: g_hat = g / rms(g),
m_hat = (m - mean(m)) / std(m).

* layers: four 3x3 "same" cross-correlations with zero padding and no bias,
  channels 2 -> 32 -> 32 -> 32 -> 1, ReLU after the first three;
* loss per image: mean((d / rms(d) - t)^2) with the target t = -s / rms(s),
  s = p_{k+1} - p_k a step taken by an optimiser; averaged over the batch;
* backward written out by hand; Adam with bias correction.
Weights are stored per layer as [C_out][C_in][3][3].
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 32, 32, 32, 1)


def layer_shapes():
    return [(CHANNELS[i + 1], CHANNELS[i], 3, 3) for i in range(4)]


def init_weights(rng):
    """He-normal initialisation, last layer scaled down so softplus(z) ~ ln 2."""
    ws = []
    for i, shp in enumerate(layer_shapes()):
        fan_in = shp[1] * 9
        w = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
        if i == 3:
            w *= 0.1
        ws.append(w)
    return ws


def conv3x3(x, w):
    """y[co, i, j] = sum_{ci, a, b} w[co, ci, a, b] x[ci, i + a - 1, j + b - 1]
    with x zero outside the image.  x: [C_in, H, W]; w: [C_out, C_in, 3, 3]."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], H, W))
    for a in range(3):
        for b in range(3):
            patch = xp[:, a:a + H, b:b + W]  # x[ci, i + a - 1, j + b - 1]
            y += np.einsum("oc,chw->ohw", w[:, :, a, b], patch)
    return y


def conv3x3_input_grad(dy, w):
    """Adjoint of conv3x3 with respect to x."""
    cout, H, W = dy.shape
    dxp = np.zeros((w.shape[1], H + 2, W + 2))
    for a in range(3):
        for b in range(3):
            dxp[:, a:a + H, b:b + W] += np.einsum("oc,ohw->chw", w[:, :, a, b], dy)
    return dxp[:, 1:-1, 1:-1]


def conv3x3_weight_grad(dy, x):
    """Gradient of sum(dy * conv3x3(x, w)) with respect to w."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((dy.shape[0], cin, 3, 3))
    for a in range(3):
        for b in range(3):
            dw[:, :, a, b] = np.einsum("ohw,chw->oc", dy, xp[:, a:a + H, b:b + W])
    return dw


def normalise_inputs(g, m):
    g = np.asarray(g, np.float64)
    m = np.asarray(m, np.float64)
    rg = np.sqrt(np.mean(g * g))
    gh = g / rg if rg > 0 else np.zeros_like(g)
    sd = m.std()
    mh = (m - m.mean()) / sd if sd > 0 else np.zeros_like(m)
    return np.stack([gh, mh])


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(ws, g, m, keep=False):
    """z [H, W], d = softplus(z) * g, and (optionally) the layer activations."""
    x = normalise_inputs(g, m)
    acts = [x]
    h = x
    for i, w in enumerate(ws):
        h = conv3x3(h, w)
        if i < 3:
            h = np.maximum(h, 0.0)
        acts.append(h)
    z = h[0]
    d = softplus(z) * np.asarray(g, np.float64)
    return (z, d, acts) if keep else (z, d)


def target(s):
    s = np.asarray(s, np.float64)
    return -s / np.sqrt(np.mean(s * s))


def loss_and_dz(z, g, t):
    """Loss mean((d/rms(d) - t)^2) for one image and its gradient in z."""
    g = np.asarray(g, np.float64)
    d = softplus(z) * g
    n = d.size
    r = np.sqrt(np.mean(d * d))
    u = d / r
    e = u - t
    loss = float(np.mean(e * e))
    dd = (2.0 / (n * r)) * (e - u * np.mean(e * u))
    return loss, dd * g * sigmoid(z)


def loss_and_grads(ws, batch):
    """Mean loss over a batch of (g, m, s) and the weight gradients."""
    total = 0.0
    grads = [np.zeros_like(w) for w in ws]
    for g, m, s in batch:
        z, d, acts = forward(ws, g, m, keep=True)
        loss, dz = loss_and_dz(z, g, target(s))
        total += loss
        dy = dz[None]
        for i in range(3, -1, -1):
            if i < 3:
                dy = dy * (acts[i + 1] > 0)
            grads[i] += conv3x3_weight_grad(dy, acts[i])
            if i > 0:
                dy = conv3x3_input_grad(dy, ws[i])
    B = len(batch)
    return total / B, [gr / B for gr in grads]


class Adam:
    def __init__(self, ws, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(w) for w in ws]
        self.v = [np.zeros_like(w) for w in ws]
        self.t = 0

    def step(self, ws, grads):
        self.t += 1
        out = []
        for i, (w, gr) in enumerate(zip(ws, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * gr
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * gr * gr
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            out.append(w - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)
