"""ctypes binding of ``libwarmnet.so`` (contract in ``include/warmnet.h``) and a 3-D U-Net on it.

Every layer runs in the HIP kernels of the library; PyTorch only provides
device memory (FP32 CUDA tensors, channels-last [n, d, h, w, c]) and the
stream.  There is no fallback: a missing library raises.

The network predicts a steady field [u_x, u_y, u_z, phi] from [mask, phi_0]
(solid mask and the initial phase field) and is trained with mean squared
error and Adam, all on the GPU.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwarmnet.so")
_lib = None


def load(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2502_12955_amd/build.py")
    lib = ct.CDLL(path)
    vp, i32, i64, f32, sz = ct.c_void_p, ct.c_int, ct.c_longlong, ct.c_float, ct.c_size_t
    lib.wn_conv3d_fwd.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp, i32, i32, i32, vp, vp]
    lib.wn_conv3d_dgrad.argtypes = [vp, i32, i32, i32, i32, i32, vp, i32, i32, vp, vp]
    lib.wn_wgrad_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32, i32]
    lib.wn_wgrad_workspace_bytes.restype = sz
    lib.wn_conv3d_wgrad.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, vp, vp, sz, vp]
    lib.wn_conv3d_wgrad_noalloc.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, vp, vp]
    lib.wn_wgrad_noalloc_max_bytes.argtypes = []
    lib.wn_wgrad_noalloc_max_bytes.restype = sz
    lib.wn_bias_grad.argtypes = [vp, i64, i32, vp, vp, sz, vp]
    lib.wn_bias_grad_workspace_bytes.argtypes = [i64, i32]
    lib.wn_bias_grad_workspace_bytes.restype = sz
    lib.wn_relu_bwd.argtypes = [vp, vp, i64, vp]
    lib.wn_add.argtypes = [vp, vp, i64, vp]
    lib.wn_add_channel.argtypes = [vp, i32, i32, vp, i32, i32, i64, vp]
    for name in ("wn_pool2_fwd", "wn_pool2_bwd", "wn_up2_fwd", "wn_up2_bwd"):
        getattr(lib, name).argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
    lib.wn_concat.argtypes = [vp, i32, vp, i32, i64, vp, vp]
    lib.wn_split.argtypes = [vp, i64, i32, i32, vp, vp, vp]
    lib.wn_mse.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp, vp]
    lib.wn_adam.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
    lib.wn_last_error.restype = ct.c_char_p
    _lib = lib
    return lib


def _p(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _ok(rc):
    if rc != 0:
        raise RuntimeError(f"warmnet error {rc}: {load().wn_last_error().decode()}")


def _stream():
    import torch

    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


# ----------------------------------------------------------------------------- layer calls
def conv3d_fwd(x, W, b, relu=False):
    n, d, h, w, ci = x.shape
    co, k = W.shape[0], W.shape[1]
    import torch

    y = torch.empty((n, d, h, w, co), dtype=torch.float32, device=x.device)
    _ok(load().wn_conv3d_fwd(_p(x), n, d, h, w, ci, _p(W), _p(b), co, k, int(relu), _p(y), _stream()))
    return y


def conv3d_dgrad(dy, W):
    n, d, h, w, co = dy.shape
    ci, k = W.shape[-1], W.shape[1]
    import torch

    dx = torch.empty((n, d, h, w, ci), dtype=torch.float32, device=dy.device)
    _ok(load().wn_conv3d_dgrad(_p(dy), n, d, h, w, co, _p(W), ci, k, _p(dx), _stream()))
    return dx


def wgrad_workspace_bytes(x_shape, co, k):
    n, d, h, w, ci = x_shape
    return load().wn_wgrad_workspace_bytes(n, d, h, w, ci, co, k)


def conv3d_wgrad(x, dy, k, dW, ws):
    n, d, h, w, ci = x.shape
    co = dy.shape[-1]
    _ok(load().wn_conv3d_wgrad(_p(x), _p(dy), n, d, h, w, ci, co, k, _p(dW), _p(ws), ws.numel() * 4, _stream()))


def conv3d_wgrad_noalloc(x, dy, k, dW):
    """Weight gradient without a workspace (the library's static scratch)."""
    n, d, h, w, ci = x.shape
    co = dy.shape[-1]
    _ok(load().wn_conv3d_wgrad_noalloc(_p(x), _p(dy), n, d, h, w, ci, co, k, _p(dW), _stream()))


def bias_grad_workspace_bytes(V, co):
    return load().wn_bias_grad_workspace_bytes(V, co)


def bias_grad(dy, db, ws=None):
    """db = sum of dy over voxels; ``ws`` a device workspace (allocated if None)."""
    import torch

    co = dy.shape[-1]
    V = dy.numel() // co
    need = bias_grad_workspace_bytes(V, co)
    if ws is None or ws.numel() * 4 < need:
        ws = torch.empty((need + 3) // 4, dtype=torch.float32, device=dy.device)
    _ok(load().wn_bias_grad(_p(dy), V, co, _p(db), _p(ws), ws.numel() * 4, _stream()))


def relu_bwd(y, g):
    _ok(load().wn_relu_bwd(_p(y), _p(g), g.numel(), _stream()))


def _resample(name, x, out_shape):
    import torch

    n, d, h, w, c = x.shape
    y = torch.empty(out_shape, dtype=torch.float32, device=x.device)
    _ok(getattr(load(), name)(_p(x), n, d, h, w, c, _p(y), _stream()))
    return y


def pool2_fwd(x):
    n, d, h, w, c = x.shape
    return _resample("wn_pool2_fwd", x, (n, d // 2, h // 2, w // 2, c))


def pool2_bwd(dy, in_shape):
    import torch

    n, d, h, w, c = in_shape
    dx = torch.empty(in_shape, dtype=torch.float32, device=dy.device)
    _ok(load().wn_pool2_bwd(_p(dy), n, d, h, w, c, _p(dx), _stream()))
    return dx


def up2_fwd(x):
    n, d, h, w, c = x.shape
    return _resample("wn_up2_fwd", x, (n, 2 * d, 2 * h, 2 * w, c))


def up2_bwd(dy):
    import torch

    n, D, H, W_, c = dy.shape
    dx = torch.empty((n, D // 2, H // 2, W_ // 2, c), dtype=torch.float32, device=dy.device)
    _ok(load().wn_up2_bwd(_p(dy), n, D // 2, H // 2, W_ // 2, c, _p(dx), _stream()))
    return dx


def concat(a, b):
    import torch

    V = a.numel() // a.shape[-1]
    y = torch.empty(a.shape[:-1] + (a.shape[-1] + b.shape[-1],), dtype=torch.float32, device=a.device)
    _ok(load().wn_concat(_p(a), a.shape[-1], _p(b), b.shape[-1], V, _p(y), _stream()))
    return y


def split(y, ca, cb):
    import torch

    V = y.numel() // y.shape[-1]
    a = torch.empty(y.shape[:-1] + (ca,), dtype=torch.float32, device=y.device)
    b = torch.empty(y.shape[:-1] + (cb,), dtype=torch.float32, device=y.device)
    _ok(load().wn_split(_p(y), V, ca, cb, _p(a), _p(b), _stream()))
    return a, b


def mse(y, t, wt=None):
    import torch

    c = y.shape[-1]
    loss = torch.empty(1, dtype=torch.float32, device=y.device)
    grad = torch.empty_like(y)
    ws = torch.empty((y.numel() + 255) // 256, dtype=torch.float32, device=y.device)
    _ok(load().wn_mse(_p(y), _p(t), _p(wt), c, y.numel(), _p(loss), _p(grad), _p(ws), _stream()))
    return loss, grad


def add_(y, x):
    """y += x in place."""
    _ok(load().wn_add(_p(x), _p(y), y.numel(), _stream()))


def add_channel_(y, jy, x, jx):
    """y[..., jy] += x[..., jx] in place (same voxel count)."""
    V = y.numel() // y.shape[-1]
    _ok(load().wn_add_channel(_p(y), y.shape[-1], jy, _p(x), x.shape[-1], jx, V, _stream()))


def adam(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    _ok(load().wn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, step, _stream()))


# ----------------------------------------------------------------------------- network
class Conv:
    """3-D convolution layer (k = 1 or 3) with bias and optional ReLU."""

    def __init__(self, ci, co, k, relu, rng, device):
        import torch

        std = np.sqrt(2.0 / (ci * k ** 3))
        w = rng.standard_normal((co, k, k, k, ci)) * std
        self.W = torch.tensor(w, dtype=torch.float32, device=device)
        self.b = torch.zeros(co, dtype=torch.float32, device=device)
        self.dW = torch.zeros_like(self.W)
        self.db = torch.zeros_like(self.b)
        self.mW, self.vW = torch.zeros_like(self.W), torch.zeros_like(self.W)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.k, self.relu, self.ci, self.co = k, relu, ci, co

    def forward(self, x):
        return conv3d_fwd(x, self.W, self.b, self.relu)

    def backward(self, x, y, dy, ws, need_dx=True):
        if self.relu:
            relu_bwd(y, dy)
        conv3d_wgrad(x, dy, self.k, self.dW, ws)
        bias_grad(dy, self.db, ws)
        return conv3d_dgrad(dy, self.W) if need_dx else None

    def params(self):
        return [(self.W, self.dW, self.mW, self.vW), (self.b, self.db, self.mb, self.vb)]


class UNet:
    """Four-level U-Net: widths (16, 32, 64, 128), two 3x3x3 convolutions per
    level, 2x average pooling down, nearest upsampling and skip concatenation
    up, a 1x1x1 head to ``cout`` channels.

    ``residual`` lists (output channel, input channel) pairs added after the
    head, so the network learns a correction to that input (for the warm
    start: the steady phase field as the initial one plus a change).  With
    ``zero_head`` the head starts at zero, so the untrained network returns
    exactly the residual inputs (the start from rest)."""

    def __init__(self, cin=2, cout=4, widths=(16, 32, 64, 128), seed=0, device="cuda:0", residual=(),
                 zero_head=False):
        rng = np.random.default_rng(seed)
        self.widths = widths
        self.enc = []
        c = cin
        for wdt in widths:
            self.enc.append((Conv(c, wdt, 3, True, rng, device), Conv(wdt, wdt, 3, True, rng, device)))
            c = wdt
        self.dec = []
        for lvl in range(len(widths) - 2, -1, -1):
            cin_d = widths[lvl + 1] + widths[lvl]
            self.dec.append((Conv(cin_d, widths[lvl], 3, True, rng, device),
                             Conv(widths[lvl], widths[lvl], 3, True, rng, device)))
        self.head = Conv(widths[0], cout, 1, False, rng, device)
        if zero_head:
            self.head.W.zero_()
        self.residual = tuple(residual)
        self.step_count = 0
        self._ws = None

    def layers(self):
        out = []
        for a, b in self.enc:
            out += [a, b]
        for a, b in self.dec:
            out += [a, b]
        return out + [self.head]

    def n_params(self):
        return sum(l.W.numel() + l.b.numel() for l in self.layers())

    def forward(self, x):
        """Returns the output and the saved activations for backward."""
        acts = {"x": x}
        skips = []
        h = x
        for lvl, (a, b) in enumerate(self.enc):
            if lvl > 0:
                acts[f"pin{lvl}"] = h
                h = pool2_fwd(h)
            acts[f"e{lvl}a_in"] = h
            h1 = a.forward(h)
            acts[f"e{lvl}a"] = h1
            h2 = b.forward(h1)
            acts[f"e{lvl}b"] = h2
            skips.append(h2)
            h = h2
        L = len(self.widths)
        for j, (a, b) in enumerate(self.dec):
            lvl = L - 2 - j
            up = up2_fwd(h)
            cat = concat(up, skips[lvl])
            acts[f"d{lvl}cat"] = cat
            h1 = a.forward(cat)
            acts[f"d{lvl}a"] = h1
            h2 = b.forward(h1)
            acts[f"d{lvl}b"] = h2
            h = h2
        acts["head_in"] = h
        y = self.head.forward(h)
        for jo, ji in self.residual:
            add_channel_(y, jo, x, ji)
        return y, acts

    def _workspace(self, acts):
        import torch

        need = 0
        for l, xin in self._layer_inputs(acts):
            need = max(need, wgrad_workspace_bytes(tuple(xin.shape), l.co, l.k),
                       bias_grad_workspace_bytes(xin.numel() // xin.shape[-1], l.co))
        if self._ws is None or self._ws.numel() * 4 < need:
            self._ws = torch.empty((need + 3) // 4, dtype=torch.float32, device=acts["x"].device)
        return self._ws

    def _layer_inputs(self, acts):
        out = []
        for lvl, (a, b) in enumerate(self.enc):
            out += [(a, acts[f"e{lvl}a_in"]), (b, acts[f"e{lvl}a"])]
        L = len(self.widths)
        for j, (a, b) in enumerate(self.dec):
            lvl = L - 2 - j
            out += [(a, acts[f"d{lvl}cat"]), (b, acts[f"d{lvl}a"])]
        return out + [(self.head, acts["head_in"])]

    def backward(self, dy, acts):
        """Accumulates nothing: every layer's dW, db are overwritten."""
        ws = self._workspace(acts)
        g = self.head.backward(acts["head_in"], None, dy, ws)
        L = len(self.widths)
        dskip = [None] * L
        for j in range(len(self.dec) - 1, -1, -1):   # decoder in reverse order: finest level first
            a, b = self.dec[j]
            lvl = L - 2 - j
            g = b.backward(acts[f"d{lvl}a"], acts[f"d{lvl}b"], g, ws)
            g = a.backward(acts[f"d{lvl}cat"], acts[f"d{lvl}a"], g, ws)
            gup, gskip = split(g, self.widths[lvl + 1], self.widths[lvl])
            dskip[lvl] = gskip
            g = up2_bwd(gup)
        for lvl in range(L - 1, -1, -1):
            a, b = self.enc[lvl]
            if dskip[lvl] is not None:
                add_(g, dskip[lvl])
            g = b.backward(acts[f"e{lvl}a"], acts[f"e{lvl}b"], g, ws)
            g = a.backward(acts[f"e{lvl}a_in"], acts[f"e{lvl}a"], g, ws, need_dx=lvl > 0)
            if lvl > 0:
                g = pool2_bwd(g, tuple(acts[f"pin{lvl}"].shape))
        return g

    def adam_step(self, lr):
        self.step_count += 1
        for l in self.layers():
            for p, g, m, v in l.params():
                adam(p, g, m, v, lr, self.step_count)

    def save(self, path):
        """Weights and biases as a plain .npz (no pickled objects)."""
        arrs = {}
        for i, l in enumerate(self.layers()):
            arrs[f"W{i}"] = l.W.cpu().numpy()
            arrs[f"b{i}"] = l.b.cpu().numpy()
        np.savez(path, widths=np.asarray(self.widths), residual=np.asarray(self.residual, dtype=np.int64).reshape(-1, 2),
                 **arrs)

    def load_params(self, path):
        """Weights and biases written by ``save`` for a network of the same shape."""
        import torch

        with np.load(path, allow_pickle=False) as z:
            if tuple(z["widths"]) != tuple(self.widths):
                raise ValueError(f"{path}: widths {tuple(z['widths'])} != {tuple(self.widths)}")
            for i, l in enumerate(self.layers()):
                W, b = z[f"W{i}"], z[f"b{i}"]
                if W.shape != tuple(l.W.shape) or b.shape != tuple(l.b.shape):
                    raise ValueError(f"{path}: layer {i} shape mismatch")
                l.W.copy_(torch.tensor(W, device=l.W.device))
                l.b.copy_(torch.tensor(b, device=l.b.device))


def conv_flops(net, shape, batch=1):
    """Multiply-add flops (x2) of one forward pass over ``batch`` samples of ``shape`` (d, h, w)."""
    V = int(np.prod(shape)) * batch
    total = 0.0
    for lvl, (a, b) in enumerate(net.enc):
        total += 2.0 * (V // 8 ** lvl) * 27 * (a.ci * a.co + b.ci * b.co)
    L = len(net.widths)
    for j, (a, b) in enumerate(net.dec):
        lvl = L - 2 - j
        total += 2.0 * (V // 8 ** lvl) * 27 * (a.ci * a.co + b.ci * b.co)
    total += 2.0 * V * net.head.ci * net.head.co
    return total


def bench(n=64, batch=2, iters=20, widths=(16, 32, 64, 128)):
    """Training-step throughput on random inputs: forward, MSE, backward, Adam."""
    import time

    import torch

    net = UNet(cin=2, cout=4, widths=widths, seed=0)
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.standard_normal((batch, n, n, n, 2)), dtype=torch.float32, device="cuda:0")
    t = torch.tensor(rng.standard_normal((batch, n, n, n, 4)), dtype=torch.float32, device="cuda:0")
    for _ in range(2):
        y, acts = net.forward(x)
        _, g = mse(y, t)
        net.backward(g, acts)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        y, acts = net.forward(x)
        _, g = mse(y, t)
        net.backward(g, acts)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    fl = 3.0 * conv_flops(net, (n, n, n), batch)
    return dict(n=n, batch=batch, ms_per_iter=dt * 1e3, conv_tflop_per_iter=fl / 1e12, tflops=fl / dt / 1e12,
                params=net.n_params())


if __name__ == "__main__":
    import json
    import sys

    print(json.dumps(bench(n=int(sys.argv[1]) if len(sys.argv) > 1 else 64)))
