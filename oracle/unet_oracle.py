"""FP64 CPU reference of the warm-start U-Net: forward pass and exact gradients.

TEST INFRASTRUCTURE ONLY.  Built from the layer oracle (``conv_oracle``);
nothing here is shared with the HIP path.  The network, for widths
(w_0 .. w_{L-1}):

    encoder level l: [pool 2x if l > 0] -> conv3 + ReLU -> conv3 + ReLU   (skip s_l)
    decoder level l = L-2 .. 0: upsample 2x -> concat [up, s_l] -> conv3 + ReLU -> conv3 + ReLU
    head: conv1 (no activation)

Parameters are a list of (W, b) in the order: encoder (two per level),
decoder (two per level, from the coarsest), head.

``rnd`` (default: none) is applied to both operands of every convolution
product, e.g. ``conv_oracle.bf16_round`` for a network whose convolutions
multiply BF16 operands; sums stay in FP64.
"""
from __future__ import annotations

import numpy as np

from . import conv_oracle as co


def _relu(x):
    return np.maximum(x, 0.0)


def _ident(a):
    return a


def forward(params, x, levels, rnd=_ident):
    """Returns the output and the cache of activations used by ``backward``."""
    it = iter(params)
    cache = {}
    h = np.asarray(x, np.float64)
    skips = []
    for lvl in range(levels):
        if lvl > 0:
            cache[("pin", lvl)] = h
            h = co.avgpool2(h)
        for j in range(2):
            W, b = next(it)
            cache[("enc_in", lvl, j)] = h
            h = _relu(co.conv3d(rnd(h), rnd(W), b))
            cache[("enc_out", lvl, j)] = h
        skips.append(h)
    for lvl in range(levels - 2, -1, -1):
        h = np.concatenate([co.upsample2(h), skips[lvl]], axis=-1)
        for j in range(2):
            W, b = next(it)
            cache[("dec_in", lvl, j)] = h
            h = _relu(co.conv3d(rnd(h), rnd(W), b))
            cache[("dec_out", lvl, j)] = h
    W, b = next(it)
    cache["head_in"] = h
    return co.conv3d(rnd(h), rnd(W), b), cache


def backward(params, cache, dy, levels, rnd=_ident):
    """Gradients (dW, db) of sum(dy * forward(params, x)) for every layer, in params order."""
    grads = [None] * len(params)
    n_enc = 2 * levels
    head = len(params) - 1
    W, _ = params[head]
    grads[head] = (co.conv3d_wgrad(rnd(cache["head_in"]), rnd(dy), W.shape[1]), co.bias_grad(dy))
    g = co.conv3d_dgrad(rnd(dy), rnd(W))

    def conv_back(idx, xin, yout, g):
        Wl, _ = params[idx]
        g = g * (yout > 0)
        grads[idx] = (co.conv3d_wgrad(rnd(xin), rnd(g), Wl.shape[1]), co.bias_grad(g))
        return co.conv3d_dgrad(rnd(g), rnd(Wl))

    dskip = [None] * levels
    idx = head - 1
    for lvl in range(0, levels - 1):      # decoder levels in reverse order of the forward pass
        for j in (1, 0):
            g = conv_back(idx, cache[("dec_in", lvl, j)], cache[("dec_out", lvl, j)], g)
            idx -= 1
        c_up = cache[("dec_in", lvl, 0)].shape[-1] - cache[("enc_out", lvl, 1)].shape[-1]
        dskip[lvl] = g[..., c_up:]
        g = co.upsample2_bwd(g[..., :c_up])
    assert idx == n_enc - 1
    for lvl in range(levels - 1, -1, -1):
        if dskip[lvl] is not None:
            g = g + dskip[lvl]
        for j in (1, 0):
            g = conv_back(2 * lvl + j, cache[("enc_in", lvl, j)], cache[("enc_out", lvl, j)], g)
        if lvl > 0:
            g = co.avgpool2_bwd(g)
    return grads, g
