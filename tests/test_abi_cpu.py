"""The C-ABI library loads on the CPU and exports every symbol the header declares (no GPU calls)."""
import ctypes as ct
import os
import re

import pytest

from paper_2502_12955_amd import inputs, mclbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mclbm.h")).read()
    return sorted(set(re.findall(r"\b(mclbm_[a-z_]+)\s*\(", src)))


def test_header_declarations_are_exported():
    lib = mclbm.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mclbm.EXPORTS)


def test_required_bytes_and_validation():
    p = inputs.porous_params(n=64)
    nb = mclbm.required_bytes(p)
    # two population buffers of 2 x 19 floats per node dominate
    assert nb > 2 * 2 * 19 * 4 * 64 ** 3
    bad = dict(p, tau=(0.5, 1.0))
    with pytest.raises(mclbm.MclbmError) as e:
        mclbm.required_bytes(bad)
    assert e.value.code == mclbm.EINVAL and "tau" in mclbm.last_error()
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, lattice="D2Q9"))      # nz != 1
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, ncomp=3))
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, D=0.0))
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, solute="inlet_outlet_x", nx=1))
    # the product species: needs the solute and D2 > 0, and adds one more set of solute planes
    nbp = mclbm.required_bytes(dict(p, product=1, D2=0.2))
    assert nbp - nb >= 2 * 7 * 4 * 64 ** 3
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, product=1, D2=0.0))
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, product=1, solute="off"))
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, product=2))
    # a per-node rate field needs the solute and adds one value per fluid node
    assert mclbm.required_bytes(dict(p, rate_field=1)) >= nb + 4 * 64 ** 3
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, rate_field=1, solute="off"))
    # particle deposition: needs the solute, DP > 0 and a single lattice; adds one FP64 deposit per node
    nbd = mclbm.required_bytes(dict(p, deposition=1, dep_prob=0.01))
    assert nbd - nb >= 8 * 64 ** 3
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, deposition=1, dep_prob=0.01, solute="off"))
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, deposition=1, dep_prob=0.0))
    with pytest.raises(mclbm.MclbmError):
        mclbm.required_bytes(dict(p, deposition=2, dep_prob=0.01))
    with pytest.raises(mclbm.MclbmError) as e:
        mclbm.required_bytes_batch([dict(p, deposition=1, dep_prob=0.01)] * 2)
    assert "single lattice" in mclbm.last_error()
    # sizes beyond the 32-bit fluid and box indexing are refused before any allocation
    with pytest.raises(mclbm.MclbmError) as e:
        mclbm.required_bytes(dict(p, nx=2048, ny=2048, nz=1024))
    assert e.value.code == mclbm.EINVAL and "32-bit" in mclbm.last_error()


def test_arena_too_small_is_rejected_before_any_device_call():
    p = inputs.droplet_2d_params(nx=16, ny=8)
    s = mclbm.params_from_dict(p)
    h = ct.c_void_p()
    rc = mclbm.load().mclbm_init_lattice(ct.byref(s), ct.c_void_p(256), 16, None, ct.byref(h))
    assert rc == mclbm.ENOMEM and not h.value


def test_warmnet_header_declarations_are_exported():
    from paper_2502_12955_amd import warmnet

    lib = warmnet.load()
    src = open(os.path.join(ROOT, "include", "warmnet.h")).read()
    names = sorted(set(re.findall(r"\b(wn_[a-z0-9_]+)\s*\(", src)))
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # argument checks happen before any device call
    assert lib.wn_conv3d_fwd(None, 1, 4, 4, 4, 2, None, None, 4, 3, 0, None, None) == -1
    assert b"bad arguments" in lib.wn_last_error()
    # 16 x 16 x 32 voxels = 32 bricks of 256; this small layer sums one brick per chunk
    assert lib.wn_wgrad_workspace_bytes(1, 16, 16, 32, 3, 5, 3) == 32 * 5 * 27 * 3 * 4
    assert lib.wn_bias_grad_workspace_bytes(ct.c_longlong(4096), 16) == 4096 // 256 * 16 * 4
