"""The no-allocation weight gradient equals the workspace one (GPU).

wn_conv3d_wgrad_noalloc keeps its chunk partial sums in the library's static
device scratch instead of a caller workspace; with the same kernels and the
same fixed-order reduction its result must equal wn_conv3d_wgrad's bit for
bit.  Two calls in a row, the second smaller, check that the scratch left by
the first call does not leak into the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _wgrad_pair(shape, co, k, seed):
    from paper_2502_12955_amd import warmnet as wn

    g = torch.Generator().manual_seed(seed)
    n, d, h, w, ci = shape
    x = torch.randn(shape, generator=g).cuda()
    dy = torch.randn((n, d, h, w, co), generator=g).cuda()
    ref = torch.empty((co, k, k, k, ci), device="cuda")
    ws = torch.empty((wn.wgrad_workspace_bytes(shape, co, k) + 3) // 4, device="cuda")
    wn.conv3d_wgrad(x, dy, k, ref, ws)
    out = torch.full_like(ref, float("nan"))
    wn.conv3d_wgrad_noalloc(x, dy, k, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_wgrad_equals_workspace_wgrad_twice():
    print("no-alloc wgrad: 2x16^3x32 -> 32 k3, then 1x8^3x16 -> 16 k3", flush=True)
    out, ref = _wgrad_pair((2, 16, 16, 16, 32), 32, 3, 1)
    assert np.array_equal(out, ref)
    out, ref = _wgrad_pair((1, 8, 8, 8, 16), 16, 3, 2)
    assert np.array_equal(out, ref)
    out, ref = _wgrad_pair((1, 8, 8, 8, 16), 4, 1, 3)
    assert np.array_equal(out, ref)


def test_noalloc_wgrad_rejects_oversized_shape():
    from paper_2502_12955_amd import warmnet as wn

    lib = wn.load()
    limit = lib.wn_wgrad_noalloc_max_bytes()
    shape = (1, 4, 4, 4, 640)   # 640 -> 640 channels: one chunk of 27 * 640^2 partials
    assert wn.wgrad_workspace_bytes(shape, 640, 3) > limit
    x = torch.zeros(1, device="cuda")
    # rejected on the host before any launch, so the 1-element tensors are never read
    rc = lib.wn_conv3d_wgrad_noalloc(wn._p(x), wn._p(x), 1, 4, 4, 4, 640, 640, 3, wn._p(x), wn._stream())
    assert rc == -1
    assert b"static scratch" in lib.wn_last_error()
