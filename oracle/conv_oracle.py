"""Plain FP64 CPU oracle of the warm-start convolutional surrogate.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

The surrogate is not part of the paper; it is a small network of four 3x3
convolutions whose definitions are written out here literally:

  layout        activations (B, H, W, C) channels-last; weights (Cout, 3, 3, Cin)
  tap (ky, kx)  reads the input at (h + (ky - 1) d, w + (kx - 1) d), zero outside
  forward       y[b,h,w,o] = bias[o] + sum_{ky,kx,i} x[b, h+(ky-1)d, w+(kx-1)d, i] W[o,ky,kx,i]
  activation    silu(y) = y / (1 + exp(-y)) after every layer but the last
  loss          L = sum_{b,h,w,c} m[b,h,w] (out - t)^2 / sum_{b,h,w} m[b,h,w]
  optimiser     Adam (Kingma & Ba) with bias correction
  pooling       mean over non-overlapping k x k blocks
  upsampling    bilinear, sample positions (i + 1/2) / k - 1/2 in coarse units,
                clamped to the edge cells
  storage       the network keeps its weights, its stored activations silu(y)
                and the gradients it propagates between layers (the loss
                gradient dL/dout and dL/dy of every hidden layer) in bf16, and
                pre-activations y in fp32; network_forward / network_backward
                take that rounding as `store` (to_bf16), or none (FP64 mode)
"""
from __future__ import annotations

import numpy as np


def conv_forward(x, W, b, d):
    B, H, Wd, Ci = x.shape
    Co = W.shape[0]
    y = np.zeros((B, H, Wd, Co)) + b[None, None, None, :]
    xp = np.zeros((B, H + 2 * d, Wd + 2 * d, Ci))
    xp[:, d:d + H, d:d + Wd] = x
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky * d:ky * d + H, kx * d:kx * d + Wd, :]          # x at (h+(ky-1)d, w+(kx-1)d)
            y += np.einsum("bhwi,oi->bhwo", patch, W[:, ky, kx, :])
    return y


def conv_backward_data(dy, W, d):
    B, H, Wd, Co = dy.shape
    Ci = W.shape[3]
    dx = np.zeros((B, H, Wd, Ci))
    dyp = np.zeros((B, H + 2 * d, Wd + 2 * d, Co))
    dyp[:, d:d + H, d:d + Wd] = dy
    for ky in range(3):
        for kx in range(3):
            # dx[h, w] += dy[h - (ky-1)d, w - (kx-1)d] W[:, ky, kx, :]
            patch = dyp[:, (2 - ky) * d:(2 - ky) * d + H, (2 - kx) * d:(2 - kx) * d + Wd, :]
            dx += np.einsum("bhwo,oi->bhwi", patch, W[:, ky, kx, :])
    return dx


def conv_backward_weight(x, dy, d):
    B, H, Wd, Ci = x.shape
    Co = dy.shape[3]
    dW = np.zeros((Co, 3, 3, Ci))
    xp = np.zeros((B, H + 2 * d, Wd + 2 * d, Ci))
    xp[:, d:d + H, d:d + Wd] = x
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky * d:ky * d + H, kx * d:kx * d + Wd, :]
            dW[:, ky, kx, :] = np.einsum("bhwo,bhwi->oi", dy, patch)
    return dW, dy.sum(axis=(0, 1, 2))


def silu(y):
    return y / (1.0 + np.exp(-y))


def silu_grad(y):
    s = 1.0 / (1.0 + np.exp(-y))
    return s * (1.0 + y * (1.0 - s))


def _identity(v):
    return v


def network_forward(x, Ws, bs, dils, store=None):
    """Returns the output and the per-layer (input, pre-activation) pairs.
    store: rounding of the stored activations silu(y) (None: exact)."""
    store = store or _identity
    a = x
    cache = []
    for l, (W, b, d) in enumerate(zip(Ws, bs, dils)):
        y = conv_forward(a, W, b, d)
        cache.append((a, y))
        a = store(silu(y)) if l < len(Ws) - 1 else y
    return a, cache


def masked_mse(out, target, mask):
    diff = out - target
    den = mask.sum()
    loss = (mask[..., None] * diff * diff).sum() / den
    dout = 2.0 * mask[..., None] * diff / den
    return loss, dout


def network_backward(dout, cache, Ws, dils, store=None):
    """Per-layer (dW, db) from dL/dout.  store: rounding of the propagated
    gradients dL/dout and dL/dy (None: exact)."""
    store = store or _identity
    grads = [None] * len(Ws)
    g = store(dout)
    for l in range(len(Ws) - 1, -1, -1):
        a, y = cache[l]
        dW, db = conv_backward_weight(a, g, dils[l])
        grads[l] = (dW, db)
        if l > 0:
            da = conv_backward_data(g, Ws[l], dils[l])
            g = store(da * silu_grad(cache[l - 1][1]))
    return grads


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def avg_pool(x, k):
    B, H, W, C = x.shape
    return x.reshape(B, H // k, k, W // k, k, C).mean(axis=(2, 4))


def upsample_bilinear(x, k):
    B, h, w, C = x.shape
    H, W = h * k, w * k

    def coords(n_fine, n_coarse):
        p = (np.arange(n_fine) + 0.5) / k - 0.5
        p = np.clip(p, 0.0, n_coarse - 1.0)
        i0 = np.floor(p).astype(int)
        i1 = np.minimum(i0 + 1, n_coarse - 1)
        return i0, i1, p - i0

    y0, y1, fy = coords(H, h)
    x0, x1, fx = coords(W, w)
    top = x[:, y0][:, :, x0] * (1 - fx)[None, None, :, None] + x[:, y0][:, :, x1] * fx[None, None, :, None]
    bot = x[:, y1][:, :, x0] * (1 - fx)[None, None, :, None] + x[:, y1][:, :, x1] * fx[None, None, :, None]
    return top * (1 - fy)[None, :, None, None] + bot * fy[None, :, None, None]


def to_bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
