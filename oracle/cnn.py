"""FP64 reference of the learned-closure network (TEST INFRASTRUCTURE ONLY).

The network corrects a coarse SMAME step: q <- S_c(q) + D f(N S_c(q)), where
f is five 3x3 convolutions (channels 3 -> 32 -> 32 -> 32 -> 32 -> 3) with
circular padding and ReLU after the first four, N and D per-channel scales.
This module computes f, its gradients and one Adam update in plain numpy
FP64, with no blocking or fusion, in the same layouts as the GPU library:

  activations  [H, W, C]                (channel fastest)
  weights      [9, C_out, C_in]          tap t = (dy + 1) * 3 + (dx + 1)
  bias         [C_out]

conv(x, w, b)[y, x, o] = b[o] + sum_{t, i} w[t, o, i] x[(y + dy) mod H, (x + dx) mod W, i]
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (3, 32, 32, 32, 32, 3)


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3 convolution with circular padding."""
    H, W, _ = x.shape
    out = np.broadcast_to(b, (H, W, w.shape[1])).astype(np.float64).copy()
    for t, (dy, dx) in enumerate(TAPS):
        xs = np.roll(x, shift=(-dy, -dx), axis=(0, 1))  # xs[y, x] = x[y + dy, x + dx]
        out += xs @ w[t].T
    return out


def conv_grads(x: np.ndarray, w: np.ndarray, g: np.ndarray):
    """Gradients of sum(g * conv(x, w, b)) with respect to x, w and b."""
    dx_ = np.zeros_like(x, dtype=np.float64)
    dw = np.zeros_like(w, dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        xs = np.roll(x, shift=(-dy, -dx), axis=(0, 1))
        dw[t] = np.einsum("hwo,hwi->oi", g, xs)
        # d/dx[y+dy, x+dx] of g[y, x] . w[t] -> shift the product back
        dx_ += np.roll(g @ w[t], shift=(dy, dx), axis=(0, 1))
    db = g.sum(axis=(0, 1))
    return dx_, dw, db


def init_params(seed: int, channels=CHANNELS, last_scale: float = 0.1):
    """He-initialised weights (seeded), zero biases; the last layer scaled
    down so the untrained correction starts small."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    nl = len(channels) - 1
    for l in range(nl):
        ci, co = channels[l], channels[l + 1]
        std = np.sqrt(2.0 / (9 * ci))
        w = rng.standard_normal((9, co, ci)) * std
        if l == nl - 1:
            w *= last_scale
        params.append([w, np.zeros(co)])
    return params


def forward(params, x0: np.ndarray):
    """Returns the raw output and the list of layer inputs (activations)."""
    acts = [x0]
    h = x0
    nl = len(params)
    for l, (w, b) in enumerate(params):
        h = conv(h, w, b)
        if l < nl - 1:
            h = np.maximum(h, 0.0)
            acts.append(h)
    return h, acts


def backward(params, acts, g_out: np.ndarray):
    """Gradients of sum(g_out * f(x0)) for every layer's (w, b)."""
    grads = [None] * len(params)
    g = g_out
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        gx, gw, gb = conv_grads(acts[l], w, g)
        grads[l] = [gw, gb]
        if l > 0:
            g = gx * (acts[l] > 0.0)  # ReLU of the layer that produced acts[l]
    return grads


def mse_loss_and_grad(raw: np.ndarray, target: np.ndarray):
    """Mean squared error over pixels and the 3 output channels."""
    d = raw - target
    n = d.size
    return float(np.sum(d * d) / n), 2.0 * d / n


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba) in place; t is the 1-based step."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)


def box_filter(f: np.ndarray, r: int) -> np.ndarray:
    """Average over r x r blocks (coarse node I covers fine nodes rI..rI+r-1)."""
    H, W = f.shape
    return f.reshape(H // r, r, W // r, r).mean(axis=(1, 3))


def prolong_bilinear(c: np.ndarray, r: int) -> np.ndarray:
    """Periodic bilinear interpolation of a coarse field onto the fine grid.
    Coarse node I sits at fine coordinate r I + (r - 1)/2."""
    Hc, Wc = c.shape
    def weights(n_f):
        s = (np.arange(n_f) - (r - 1) / 2.0) / r
        i0 = np.floor(s).astype(int)
        t = s - i0
        return i0, t
    iy, ty = weights(Hc * r)
    ix, tx = weights(Wc * r)
    y0, y1 = iy % Hc, (iy + 1) % Hc
    x0, x1 = ix % Wc, (ix + 1) % Wc
    a = c[y0][:, x0] * (1 - tx)[None, :] + c[y0][:, x1] * tx[None, :]
    b = c[y1][:, x0] * (1 - tx)[None, :] + c[y1][:, x1] * tx[None, :]
    return a * (1 - ty)[:, None] + b * ty[:, None]
