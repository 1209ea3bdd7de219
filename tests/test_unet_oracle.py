"""Pins of the U-Net oracle (no GPU): its gradients against central finite differences."""
import numpy as np

from oracle import unet_oracle as uo


def _params(widths, cin, cout, seed):
    rng = np.random.default_rng(seed)
    shapes = []
    c = cin
    for w in widths:
        shapes += [(w, 3, c), (w, 3, w)]
        c = w
    for lvl in range(len(widths) - 2, -1, -1):
        shapes += [(widths[lvl], 3, widths[lvl + 1] + widths[lvl]), (widths[lvl], 3, widths[lvl])]
    shapes.append((cout, 1, widths[0]))
    return [(rng.standard_normal((o, k, k, k, i)) * np.sqrt(2.0 / (i * k ** 3)), 0.1 * rng.standard_normal(o))
            for o, k, i in shapes]


def test_gradients_match_finite_differences():
    widths, levels = (2, 3, 4), 3
    params = _params(widths, 2, 3, 0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 8, 8, 8, 2))
    dy = rng.standard_normal((1, 8, 8, 8, 3))
    y, cache = uo.forward(params, x, levels)
    assert y.shape == (1, 8, 8, 8, 3)
    grads, dx = uo.backward(params, cache, dy, levels)
    dirs = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    dxd = rng.standard_normal(x.shape)
    eps = 1e-6

    def loss(s):
        p = [(W + s * dW, b + s * db) for (W, b), (dW, db) in zip(params, dirs)]
        return np.sum(dy * uo.forward(p, x + s * dxd, levels)[0])

    fd = (loss(eps) - loss(-eps)) / (2 * eps)
    an = sum(np.sum(gW * dW) + np.sum(gb * db) for (gW, gb), (dW, db) in zip(grads, dirs)) + np.sum(dx * dxd)
    assert abs(fd - an) < 1e-6 * abs(an)
    # each layer separately, so that a wrong gradient cannot hide behind a sum
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        dW = rng.standard_normal(W.shape)

        def loss_i(s):
            p = list(params)
            p[i] = (W + s * dW, b)
            return np.sum(dy * uo.forward(p, x, levels)[0])

        fd = (loss_i(eps) - loss_i(-eps)) / (2 * eps)
        assert abs(fd - np.sum(gW * dW)) < 1e-6 * max(1.0, abs(fd)), i
