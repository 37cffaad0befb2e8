"""Learned warm start network, plain FP64 NumPy (test infrastructure only).

x0 = A^H b + f(A^H b), where f is five 3x3 convolutions with "same" zero
padding, channels 2 -> 32 -> 32 -> 32 -> 32 -> 2, ReLU after the first four,
applied to the real and imaginary parts of the zero-filled image (NHWC,
channel 0 = real, 1 = imaginary).  FIRLS then starts from x0 (the start
point of Algorithms 2 and 3 is free; Section 3.3 uses A^H b).

``bf16=True`` rounds, exactly where the GPU stores bfloat16, the network
input, every weight tensor, every hidden activation and every gradient fed
to a product, to the nearest bfloat16 (ties to even); sums stay in FP64.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 32, 32, 32, 32, 2)


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) via float32, returned as
    float64.  Finite inputs only."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def init_params(seed: int = 0):
    """He-normal weights [3, 3, Cin, Cout], zero biases; the last layer is
    scaled by 0.1 so that the untrained network starts near x0 = A^H b."""
    rs = np.random.default_rng(np.random.SeedSequence([int(seed), 17]))
    params = []
    for i in range(5):
        cin, cout = CHANNELS[i], CHANNELS[i + 1]
        W = rs.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / (9 * cin))
        if i == 4:
            W *= 0.1
        params.append((W.astype(np.float32).astype(np.float64), np.zeros(cout)))
    return params


def conv3x3(x, W, b):
    """y[n,i,j,o] = sum_{dy,dx,c} x[n, i+dy-1, j+dx-1, c] W[dy,dx,c,o] + b[o]
    with zeros outside the image."""
    n, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((n, H, Wd, W.shape[3]))
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + Wd, :] @ W[dy, dx]
    return y + b


def conv3x3_backward(x, W, gy):
    """Gradients of sum(gy * conv3x3(x, W, b)) with respect to x, W, b."""
    n, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            gxp[:, dy:dy + H, dx:dx + Wd, :] += gy @ W[dy, dx].T
            gW[dy, dx] = np.einsum("nhwc,nhwo->co", xp[:, dy:dy + H, dx:dx + Wd, :], gy)
    return gxp[:, 1:H + 1, 1:Wd + 1, :], gW, gy.sum(axis=(0, 1, 2))


def to_channels(z):
    """Complex [n, H, W] -> real [n, H, W, 2]."""
    return np.stack([z.real, z.imag], axis=-1)


def from_channels(a):
    return a[..., 0] + 1j * a[..., 1]


def forward(params, zf, bf16_mode: bool = False):
    """x0 for a batch of zero-filled images zf (complex [n, H, W]).
    Returns (x0 complex [n, H, W], cache for backward)."""
    rnd = bf16 if bf16_mode else (lambda a: a)
    h = rnd(to_channels(zf))
    acts = [h]
    Ws = [rnd(W) for W, _ in params]
    for i in range(5):
        y = conv3x3(h, Ws[i], params[i][1])
        if i < 4:
            h = rnd(np.maximum(y, 0.0))
            acts.append(h)
        else:
            out = y
    x0 = zf + from_channels(out)
    return x0, {"acts": acts, "Ws": Ws, "bf16": bf16_mode}


def loss(x0, label):
    """Mean squared error over pixels and the two channels."""
    d = to_channels(x0 - label)
    return float(np.mean(d * d))


def loss_grad(x0, label):
    """d loss / d x0 as real [n, H, W, 2]."""
    d = to_channels(x0 - label)
    return 2.0 * d / d.size


def backward(cache, g_out):
    """Gradients of the loss with respect to every (W, b), given
    g_out = d loss / d (network output) as real [n, H, W, 2]."""
    rnd = bf16 if cache["bf16"] else (lambda a: a)
    acts, Ws = cache["acts"], cache["Ws"]
    grads = [None] * 5
    g = rnd(g_out)
    for i in range(4, -1, -1):
        gx, gW, gb = conv3x3_backward(acts[i], Ws[i], g)
        grads[i] = (gW, gb)
        if i > 0:
            g = rnd(gx * (acts[i] > 0.0))
    return grads


def adam(param, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), bias-corrected; returns new (param, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v
