"""FP64 CPU reference for the warm-start network's layers.

TEST INFRASTRUCTURE ONLY (tests and the benchmark's baseline leg).  Plain
numpy, shares nothing with the HIP kernels.  Tensors are channels-last
[n, d, h, w, c]; convolution weights are [c_out, kz, ky, kx, c_in] with odd
cubic kernels (1 or 3) and periodic (circular) padding, matching the
periodic lattice the network is trained on.

    conv3d(x, W, b)[n, z, y, x, o] = b[o] + sum_{k, i} W[o, k, i] x[n, p + k - r, i]
    conv3d_dgrad = adjoint of conv3d with respect to x
    conv3d_wgrad = derivative of sum(dy * conv3d(x, W)) with respect to W
    avgpool2 / upsample2 (nearest) and their adjoints
"""
from __future__ import annotations

import numpy as np


def _shifted(x, dz, dy, dx):
    """x[n, z + dz, y + dy, x + dx, c] with periodic wrap."""
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def conv3d(x, W, b=None):
    x = np.asarray(x, np.float64)
    W = np.asarray(W, np.float64)
    co, kd, kh, kw, ci = W.shape
    r = kd // 2
    out = np.zeros(x.shape[:4] + (co,))
    for a in range(kd):
        for bb in range(kh):
            for c in range(kw):
                xs = _shifted(x, a - r, bb - r, c - r)
                out += xs @ W[:, a, bb, c, :].T
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3d_dgrad(dy, W):
    dy = np.asarray(dy, np.float64)
    W = np.asarray(W, np.float64)
    co, kd, kh, kw, ci = W.shape
    r = kd // 2
    dx = np.zeros(dy.shape[:4] + (ci,))
    for a in range(kd):
        for bb in range(kh):
            for c in range(kw):
                dx += _shifted(dy, r - a, r - bb, r - c) @ W[:, a, bb, c, :]
    return dx


def conv3d_wgrad(x, dy, k):
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    r = k // 2
    ci, co = x.shape[-1], dy.shape[-1]
    dW = np.zeros((co, k, k, k, ci))
    X = x.reshape(-1, ci)
    for a in range(k):
        for bb in range(k):
            for c in range(k):
                xs = _shifted(x, a - r, bb - r, c - r).reshape(-1, ci)
                dW[:, a, bb, c, :] = dy.reshape(-1, co).T @ xs
    return dW


def bias_grad(dy):
    return np.asarray(dy, np.float64).reshape(-1, dy.shape[-1]).sum(axis=0)


def avgpool2(x):
    n, d, h, w, c = x.shape
    return np.asarray(x, np.float64).reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def avgpool2_bwd(dy):
    return np.repeat(np.repeat(np.repeat(np.asarray(dy, np.float64), 2, 1), 2, 2), 2, 3) / 8.0


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(np.asarray(x, np.float64), 2, 1), 2, 2), 2, 3)


def upsample2_bwd(dy):
    n, d, h, w, c = dy.shape
    return np.asarray(dy, np.float64).reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def bf16_round(a):
    """Round FP32 values to BF16 (nearest even) and back, as the MFMA operands see them."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def mse(y, t, wt=None):
    """Loss mean(wt[c] (y - t)^2) over all values and its gradient with respect to y."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    w = np.ones(y.shape[-1]) if wt is None else np.asarray(wt, np.float64)
    e = y - t
    return float(np.mean(w * e * e)), 2.0 * w * e / e.size


def adam(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One step of Adam (Kingma and Ba, Algorithm 1): returns the new (p, m, v)."""
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * np.asarray(g, np.float64)
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * np.asarray(g, np.float64) ** 2
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return np.asarray(p, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v
