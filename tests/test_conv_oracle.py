"""Pins of the network-layer oracle (no GPU): library special cases and exact adjoint identities."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import conv_oracle as co


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_delta_kernel_is_a_periodic_shift():
    x = _rand((2, 5, 6, 7, 3), 0)
    W = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        W[c, 2, 0, 1, c] = 1.0           # picks x[z + 1, y - 1, x]
    y = co.conv3d(x, W)
    assert np.array_equal(y, np.roll(x, shift=(-1, 1, 0), axis=(1, 2, 3)))


def test_single_channel_matches_scipy_correlate_wrap():
    x = _rand((1, 6, 7, 8, 1), 1)
    k = _rand((3, 3, 3), 2)
    y = co.conv3d(x, k[None, :, :, :, None], b=[0.25])
    ref = ndimage.correlate(x[0, :, :, :, 0], k, mode="wrap") + 0.25
    assert np.max(np.abs(y[0, :, :, :, 0] - ref)) < 1e-12


@pytest.mark.parametrize("k", [1, 3])
def test_dgrad_is_the_adjoint(k):
    x = _rand((2, 4, 5, 6, 3), 3)
    W = _rand((4, k, k, k, 3), 4)
    dy = _rand((2, 4, 5, 6, 4), 5)
    lhs = np.sum(co.conv3d(x, W) * dy)
    rhs = np.sum(x * co.conv3d_dgrad(dy, W))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


@pytest.mark.parametrize("k", [1, 3])
def test_wgrad_is_the_weight_derivative(k):
    x = _rand((1, 4, 6, 5, 3), 6)
    dy = _rand((1, 4, 6, 5, 2), 7)
    V = _rand((2, k, k, k, 3), 8)
    lhs = np.sum(dy * co.conv3d(x, V))
    rhs = np.sum(co.conv3d_wgrad(x, dy, k) * V)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    assert np.allclose(co.bias_grad(dy), dy.sum(axis=(0, 1, 2, 3)))


def test_pool_and_upsample_adjoints():
    x = _rand((2, 4, 6, 8, 3), 9)
    y = _rand((2, 2, 3, 4, 3), 10)
    assert abs(np.sum(co.avgpool2(x) * y) - np.sum(x * co.avgpool2_bwd(y))) < 1e-12
    assert abs(np.sum(co.upsample2(y) * x) - np.sum(y * co.upsample2_bwd(x))) < 1e-12
    assert np.allclose(co.avgpool2(co.upsample2(y)), y)


def test_bf16_rounding_matches_torch():
    import torch

    v = np.concatenate([_rand(1000, 11).astype(np.float32),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 1e-30], np.float32)])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(co.bf16_round(v), ref)


def test_mse_gradient_by_finite_difference():
    y = _rand((2, 3, 4, 4, 3), 12)
    t = _rand((2, 3, 4, 4, 3), 13)
    wt = [1.0, 0.5, 2.0]
    loss, g = co.mse(y, t, wt)
    assert abs(loss - np.sum(np.array(wt) * (y - t) ** 2) / y.size) < 1e-14
    d = _rand(y.shape, 14)
    eps = 1e-6
    fd = (co.mse(y + eps * d, t, wt)[0] - co.mse(y - eps * d, t, wt)[0]) / (2 * eps)
    assert abs(fd - np.sum(g * d)) < 1e-8


def test_adam_first_step_is_lr_times_sign():
    # with zero moments the bias-corrected first step is lr g / (|g| + eps)
    g = np.array([3.0, -0.02, 1e-3, -7.0])
    p, m, v = co.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), lr=0.01, step=1, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps the step at lr for every later step
    for s in range(2, 6):
        p, m, v = co.adam(p, g, m, v, lr=0.01, step=s, eps=0.0)
    assert np.allclose(p, -0.05 * np.sign(g), rtol=1e-12, atol=0)
