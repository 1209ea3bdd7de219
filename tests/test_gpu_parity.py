"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

FP64 storage: every value within 1e-12 of its field's scale, max|a - b| <=
1e-12 max|b| per field (the method is deterministic; only summation order
differs).  FP32: one step from the same
state, per-value error <= 2e-6 of the population scale.  Geometry and link
masks: bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs

from helpers import gpu_lattice, maxrel, oracle_state, small_porous, split_pops

pytestmark = pytest.mark.gpu

BLOCKS = [256, 64]


@pytest.fixture(scope="module")
def variants():
    """Launch shapes exercised by the parity tests (results must not depend on them)."""
    return BLOCKS


@pytest.mark.parametrize("forcing", ["guo", "sc"])
def test_droplet_2d_fp64_matches_oracle_over_2000_steps(forcing, variants):
    """D2Q9 two-component droplet, 128x64, tau = 1, G_c = 5, 2000 steps, both forcings."""
    p, mask, rho, _, _ = inputs.droplet_2d_case(forcing=forcing)
    m, f, h = oracle_state(p, mask, rho)
    ref = []
    for _ in range(4):
        oracle.step(p, m, f, h, 500)
        ref.append(oracle.moments(p, m, f, h))
    for var in variants:
        lat = gpu_lattice(p, mask, rho, block=var)
        for k in range(4):
            lat.step(500)
            r, u, _ = lat.moments()
            print(var, (k + 1) * 500, maxrel(r, ref[k][0]), maxrel(u, ref[k][1]), flush=True)
            assert maxrel(r, ref[k][0]) < 1e-12
            assert maxrel(u, ref[k][1]) < 1e-12
        mon = lat.monitors()
        assert mon[0] == 2000
        rr = ref[-1][0]
        assert abs(mon[1] - rr[0].sum()) < 1e-12 * rr[0].sum()
        assert abs(mon[2] - rr[1].sum()) < 1e-12 * rr[1].sum()
        lat.close()


@pytest.mark.parametrize("forcing", ["guo", "sc"])
@pytest.mark.parametrize("solute", ["inlet_outlet_x", "periodic"])
def test_porous_3d_fp64_populations_match_oracle(forcing, solute, variants):
    """D3Q19 x2 + D3Q7, sphere pack with ragged box sizes, adhesion, drive, wall
    reaction; every population after 200 steps."""
    p, mask, rho, u, C = small_porous(forcing=forcing, solute=solute, storage="f64",
                                      tau=(0.9, 1.3) if forcing == "sc" else (1.0, 1.0),
                                      k_wall=0.05, C_in=1.0)
    m, f, h = oracle_state(p, mask, rho, u, C)
    oracle.step(p, m, f, h, 200)
    for var in variants:
        lat = gpu_lattice(p, mask, rho, u, C, block=var)
        lat.step(200)
        fg, hg = split_pops(p, lat.populations())
        print(var, forcing, solute, maxrel(fg, f), maxrel(hg, h), flush=True)
        assert maxrel(fg, f) < 1e-12
        assert maxrel(hg, h) < 1e-12
        lat.close()


def test_single_component_channel_2d_with_solute(variants):
    """One component, D2Q9 + D2Q5, walls, body force, reactive walls, inlet/outlet."""
    nx, ny = 33, 17
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=ny, nz=1, ncomp=1, G=((0, 0), (0, 0)),
                           G_ads=(0.0, 0.0), accel=(2e-5, 0, 0), solute="inlet_outlet_x", D=0.2,
                           J0=0.4, k_wall=0.02, C_in=0.9, storage="f64", tau=(0.8, 0.8))
    mask = np.zeros((1, ny, nx), np.uint8)
    mask[0, 0, :] = 1
    mask[0, ny - 1, :] = 1
    mask[0, 6:10, 12:15] = 1
    rho = np.where(mask == 0, 1.0, 0.0)[None]
    m, f, h = oracle_state(p, mask, rho)
    oracle.step(p, m, f, h, 300)
    for var in variants:
        lat = gpu_lattice(p, mask, rho, block=var)
        lat.step(300)
        fg, hg = split_pops(p, lat.populations())
        assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12
        lat.close()


def test_geometry_and_links_bit_exact():
    """Pinch-fill result and link masks identical to the oracle's (sphere pack 64^3)."""
    p, mask, _, _, _ = inputs.porous_case(shape=(64, 64, 64), porosity=0.4, radius=8)
    from paper_2502_12955_amd import mclbm
    lat = mclbm.Lattice(p)
    n = lat.set_geometry(mask)
    gm, gfb, gsb = lat.get_geometry()
    om, on = oracle.pinch_fill(p, mask)
    ofb, osb = oracle.link_masks(p, om)
    assert n == on
    assert np.array_equal(gm, om.reshape(-1))
    assert np.array_equal(gfb, ofb)
    assert np.array_equal(gsb, osb)
    lat.close()


def test_fp32_one_step_matches_oracle_from_same_state(variants):
    """FP32 path vs the FP64 oracle from the identical (FP32-representable) state."""
    p, mask, rho, u, C = small_porous(storage="f32", k_wall=0.05, C_in=1.0)
    for var in variants:
        lat = gpu_lattice(p, mask, rho, u, C, block=var)
        lat.step(7)
        pops = lat.populations()
        fs, hs = split_pops(p, pops)
        m, _ = oracle.pinch_fill(p, mask)
        f64, h64 = fs.copy(), hs.copy()
        oracle.step(p, m, f64, h64, 1)
        lat.step(1)
        fg, hg = split_pops(p, lat.populations())
        scale = np.abs(f64).max()
        print(var, np.abs(fg - f64).max() / scale, np.abs(hg - h64).max(), flush=True)
        assert np.abs(fg - f64).max() < 2e-6 * scale
        assert np.abs(hg - h64).max() < 2e-6 * max(1.0, np.abs(h64).max())
        lat.close()


def test_checkpoint_resume_and_determinism(variants):
    p, mask, rho, u, C = small_porous(storage="f32", k_wall=0.05, C_in=1.0)
    for var in variants:
        a = gpu_lattice(p, mask, rho, u, C, block=var)
        a.step(10)
        snap = a.populations(raw=True)
        a.step(15)
        end_a = a.populations(raw=True)
        b = gpu_lattice(p, mask, rho, u, C, block=var)
        b.step(10)
        b.set_populations(snap, raw=True)
        b.step(15)
        assert np.array_equal(b.populations(raw=True), end_a)   # resume is bit-exact
        c = gpu_lattice(p, mask, rho, u, C, block=var)
        c.step(25)
        assert np.array_equal(c.populations(raw=True), end_a)   # runs are deterministic
        for x in (a, b, c):
            x.close()


def test_launch_shapes_agree_bitwise():
    """Every fluid node is updated by one thread with the same arithmetic, so the
    workgroup size cannot change a single bit."""
    p, mask, rho, u, C = small_porous(storage="f32", k_wall=0.05, C_in=1.0)
    out = []
    for bs in (64, 128, 256):
        lat = gpu_lattice(p, mask, rho, u, C, block=bs)
        lat.step(20)
        out.append(lat.populations(raw=True))
        lat.close()
    assert all(np.array_equal(out[0], o) for o in out[1:])


def test_monitors_match_oracle():
    p, mask, rho, u, C = small_porous(storage="f64", k_wall=0.05, C_in=1.0, monitor_every=10)
    m, f, h = oracle_state(p, mask, rho, u, C)
    lat = gpu_lattice(p, mask, rho, u, C)
    lat.step(10)
    mon = lat.monitors()
    assert mon[0] == 10 and np.isinf(mon[4])
    oracle.step(p, m, f, h, 10)
    r1, u1, C1 = oracle.moments(p, m, f, h)
    lat.step(10)
    mon = lat.monitors()
    oracle.step(p, m, f, h, 10)
    r2, u2, C2 = oracle.moments(p, m, f, h)
    fluid = m.reshape(-1) == 0
    assert abs(mon[1] - r2[0].sum()) < 1e-12 * r2[0].sum()
    assert abs(mon[2] - r2[1].sum()) < 1e-12 * r2[1].sum()
    assert abs(mon[3] - C2.sum()) < 1e-12 * C2.sum()
    assert abs(mon[4] - oracle.residual(u2, u1, fluid)) < 1e-9 * oracle.residual(u2, u1, fluid)
    ph1, ph2 = oracle.phase_field(r1), oracle.phase_field(r2)
    assert abs(mon[5] - oracle.residual(ph2, ph1, fluid)) < 1e-9 * oracle.residual(ph2, ph1, fluid)
    assert abs(mon[6] - oracle.residual(C2, C1, fluid)) < 1e-9 * oracle.residual(C2, C1, fluid)
    assert mon[7] == 0 and mon[8] == fluid.sum()
    lat.close()


def test_errors_and_state_checks():
    from paper_2502_12955_amd import mclbm
    p, mask, rho, _, _ = inputs.droplet_2d_case(nx=16, ny=8, radius=3)
    lat = mclbm.Lattice(p)
    with pytest.raises(mclbm.MclbmError) as e:
        lat.step(1)
    assert e.value.code == mclbm.ESTATE
    with pytest.raises(mclbm.MclbmError) as e:
        lat.set_geometry(np.ones((1, 8, 16), np.uint8))
    assert e.value.code == mclbm.EINVAL
    lat.set_geometry(mask)
    with pytest.raises(mclbm.MclbmError) as e:
        lat.init_fields(np.zeros_like(rho))
    assert e.value.code == mclbm.EINVAL
    lat.init_fields(rho)
    pops = lat.populations()
    pops[5] = np.nan
    lat.set_populations(pops)
    lat.monitor_now(allow_diverged=True)
    assert lat.monitors()[7] >= 1
    with pytest.raises(mclbm.MclbmError) as e:
        lat.monitor_now()
    assert e.value.code == mclbm.EDIVERGED
    lat.close()
