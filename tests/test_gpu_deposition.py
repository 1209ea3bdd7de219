"""GPU: particle deposition (sec:particle_deposition, eq:surface_deposition) against
the FP64 oracle, through the C ABI.

The deposits grow at the nodes next to the substrate after every step, nodes
whose deposit exceeds 1 turn solid (the pinch rule again), and the run goes on
on the new geometry.  After many conversions the solid mask is bit-identical to
the oracle's, the populations and deposits agree element by element to 1e-12
of each field's scale, and the count of converted nodes matches.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs, mclbm

from helpers import maxrel, split_pops

pytestmark = pytest.mark.gpu


def _case(lattice, ncomp, shape, sample, **kw):
    p, mask, rho, _, _ = inputs.porous_case(shape=shape, porosity=0.6, radius=3, blob_radius=2, sample=sample)
    p.update(lattice=lattice, nz=shape[0], ncomp=ncomp, solute="inlet_outlet_x", C_in=1.0, k_wall=0.02, D=0.2,
             accel=(2e-5, 0.0, 0.0), storage="f64", deposition=1, dep_prob=0.02, monitor_every=50)
    if ncomp == 1:
        p["G"] = ((0.0, 0.0), (0.0, 0.0))
        rho = np.where(mask == 0, 1.0, 0.0)[None]
    p.update(kw)
    C = 0.2 * np.ones(shape)
    return p, mask, rho, C


def _run_both(p, mask, rho, C, steps, k_node=None):
    po = dict(p) if k_node is None else dict(p, k_node=k_node)
    m, _ = oracle.pinch_fill(po, mask)
    m = np.ascontiguousarray(m.reshape(-1))
    f, h = oracle.init(po, m, rho, None, C)
    Cps = np.zeros(m.size)
    conv = oracle.step_deposit(po, m, f, h, Cps, p["dep_prob"], steps)
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    if k_node is not None:
        lat.set_wall_rate(k_node)
    lat.init_fields(rho, None, C)
    lat.step(steps)
    return (m, f, h, Cps, conv), lat


@pytest.mark.parametrize("lattice,ncomp,shape", [("D2Q9", 1, (1, 40, 48)), ("D2Q9", 2, (1, 36, 40)),
                                                 ("D3Q19", 2, (12, 14, 18))])
def test_deposition_matches_oracle(lattice, ncomp, shape):
    p, mask, rho, C = _case(lattice, ncomp, shape, sample=5)
    (m, f, h, Cps, conv), lat = _run_both(p, mask, rho, C, 160)
    mg, _, _ = lat.get_geometry()
    fg, hg = split_pops(p, lat.populations())
    Cg, convg = lat.get_deposit()
    print(lattice, ncomp, conv, convg, maxrel(fg, f), maxrel(hg, h), maxrel(Cg, Cps), flush=True)
    assert conv > 10                                  # several conversions happened
    assert np.array_equal(mg, m)
    assert convg == conv
    assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12
    assert maxrel(Cg, Cps) < 1e-12
    assert np.all(Cg[m != 0] == 0.0)
    # monitors count the fluid nodes of the new geometry
    lat.monitor_now()
    assert lat.monitors()[8] == int((m == 0).sum())
    lat.close()


@pytest.mark.parametrize("storage", ["f16s", "bf16s", "f32"])
def test_renumbering_keeps_the_values_of_surviving_nodes(storage):
    """Two components (the paired 16-bit layout, and FP32 planes): at the step
    where nodes turn solid, every node that stays fluid holds exactly the
    populations that the same step gives without deposition (a handle with
    deposition off, started from the same state on the same geometry), and the
    mask only gains solid nodes."""
    p, mask, rho, C = _case("D2Q9", 2, (1, 36, 40), sample=7, storage=storage, dep_prob=0.05)
    # uniform component densities: the 16-bit storage shift (the mean initial density
    # over the fluid nodes) is then the same for the reference handle, set up on the
    # geometry after some conversions, and the stored bits compare directly
    fl = (mask == 0).astype(np.float64)
    rho = np.stack([0.7 * fl, 0.3 * fl])
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    lat.init_fields(rho, None, C)
    q = dict(p, deposition=0, dep_prob=0.0)
    checked = 0
    for _ in range(400):
        m0, _, _ = lat.get_geometry()
        pops0 = lat.populations(raw=True)
        conv0 = lat.get_deposit()[1]
        lat.step(1)
        m1, _, _ = lat.get_geometry()
        conv1 = lat.get_deposit()[1]
        if conv1 == conv0:
            continue
        ref = mclbm.Lattice(q)
        ref.set_geometry(m0)
        ref.init_fields(rho, None, C)
        ref.set_populations(pops0, raw=True)
        ref.step(1)
        want = ref.populations(raw=True).reshape(-1, m1.size)
        ref.close()
        got = lat.populations(raw=True).reshape(-1, m1.size)
        fluid = m1.reshape(-1) == 0
        assert np.array_equal(got[:, fluid], want[:, fluid])
        assert np.all(m1.reshape(-1) >= m0.reshape(-1)) and np.count_nonzero(m1 != m0) >= conv1 - conv0
        checked += 1
        if checked == 3:
            break
    lat.close()
    print(storage, "conversions checked", checked, flush=True)
    assert checked >= 1


def test_deposition_keeps_the_rate_field_across_rebuilds():
    p, mask, rho, C = _case("D2Q9", 1, (1, 32, 40), sample=6, rate_field=1, k_wall=0.0)
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in mask.shape], indexing="ij")
    k_node = inputs.arrhenius_rate_field(700.0 + 10.0 * xx + 3.0 * yy, 1.0, 2500.0).reshape(-1)
    (m, f, h, Cps, conv), lat = _run_both(p, mask, rho, C, 150, k_node=k_node)
    mg, _, _ = lat.get_geometry()
    fg, hg = split_pops(p, lat.populations())
    Cg, convg = lat.get_deposit()
    print(conv, convg, maxrel(hg, h), flush=True)
    assert conv > 10 and convg == conv and np.array_equal(mg, m)
    assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12 and maxrel(Cg, Cps) < 1e-12
    lat.close()


def test_deposition_in_fp32_tracks_the_fp64_oracle():
    """FP32 storage decides the conversions in its own precision: the masks agree
    up to a few nodes whose deposit sits at the threshold."""
    p, mask, rho, C = _case("D2Q9", 1, (1, 40, 48), sample=5, storage="f32")
    (m, f, h, Cps, conv), lat = _run_both(p, mask, rho, C, 160)
    mg, _, _ = lat.get_geometry()
    _, convg = lat.get_deposit()
    print(conv, convg, int((mg != m).sum()), flush=True)
    assert conv > 10
    assert int((mg != m).sum()) <= max(2, conv // 50)
    lat.close()


def test_deposit_calls_check_their_state():
    p, mask, rho, C = _case("D2Q9", 1, (1, 16, 20), sample=7)
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    with pytest.raises(mclbm.MclbmError) as e:
        lat.get_deposit()
    assert e.value.code == mclbm.ESTATE
    lat.init_fields(rho, None, C)
    Cg, n = lat.get_deposit()
    assert n == 0 and np.all(Cg == 0.0)
    lat.close()
    q = dict(p, deposition=0)
    lat = mclbm.Lattice(q)
    lat.set_geometry(mask)
    lat.init_fields(rho, None, C)
    with pytest.raises(mclbm.MclbmError) as e:
        lat.get_deposit()
    assert e.value.code == mclbm.EINVAL
    lat.close()


def test_a_channel_that_fills_up_is_reported():
    """Three fluid rows between two walls at rest with a uniform particle fraction:
    the rows next to the walls turn solid after exactly 271 steps (the oracle's closed
    form for DP c0 = 0.0037) and the middle row is then pinched, so no fluid is left:
    the step that does it fails with EINVAL and says why."""
    nz, ny, nx = 1, 5, 12
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=ny, nz=nz, ncomp=1, G=((0, 0), (0, 0)), tau=(0.8, 0.8),
                           solute="periodic", D=0.15, J0=0.2, k_wall=0.0, storage="f64", deposition=1,
                           dep_prob=0.01)
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[0, 0, :] = 1
    mask[0, ny - 1, :] = 1
    rho = np.where(mask == 0, 1.0, 0.0)[None]
    C = np.where(mask == 0, 0.37, 0.0)
    m = mask.reshape(-1).copy()                        # the oracle updates its mask in place
    f, h = oracle.init(p, m, rho, None, C)
    Cps = np.zeros(m.size)
    assert oracle.step_deposit(p, m, f, h, Cps, 0.01, 270) == 0
    Cps270 = Cps.copy()
    assert oracle.step_deposit(p, m, f, h, Cps, 0.01, 1) == 3 * nx and m.all()
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    lat.init_fields(rho, None, C)
    lat.step(270)
    Cg, conv = lat.get_deposit()
    assert conv == 0 and maxrel(Cg, Cps270) < 1e-12
    with pytest.raises(mclbm.MclbmError) as e:
        lat.step(5)
    assert e.value.code == mclbm.EINVAL and "no fluid node" in str(e.value)
    lat.close()


def test_a_deposition_run_resumes_bit_for_bit_from_a_checkpoint():
    """Checkpoint after conversions (solid mask, raw populations, deposits), restore
    into a new lattice, and both continue through further conversions identically."""
    p, mask, rho, C = _case("D2Q9", 2, (1, 36, 40), sample=5)
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    lat.init_fields(rho, None, C)
    lat.step(90)
    m90, _, _ = lat.get_geometry()
    pops = lat.populations(raw=True)
    Cps, conv = lat.get_deposit()
    assert conv > 0
    lat.step(70)
    lat2 = mclbm.Lattice(p)
    lat2.set_geometry(m90)
    lat2.init_fields(rho * (m90.reshape(mask.shape) == 0), None, C)
    lat2.set_populations(pops, raw=True)
    lat2.set_deposit(Cps, conv)
    lat2.step(70)
    a, b = lat.get_deposit(), lat2.get_deposit()
    print(conv, a[1], b[1], flush=True)
    assert a[1] == b[1] and a[1] > conv
    assert np.array_equal(lat.get_geometry()[0], lat2.get_geometry()[0])
    assert np.array_equal(lat.populations(raw=True), lat2.populations(raw=True))
    assert np.array_equal(a[0], b[0])
    lat.close()
    lat2.close()


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_deposition_with_16_bit_storage_resumes_bit_for_bit(storage):
    """16-bit shifted storage: conversions happen, the state stays finite, and a
    restored checkpoint continues bit for bit (the renumbering moves 2-byte values)."""
    p, mask, rho, C = _case("D2Q9", 1, (1, 40, 48), sample=5, storage=storage)
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    lat.init_fields(rho, None, C)
    lat.step(100)
    m100, _, _ = lat.get_geometry()
    pops = lat.populations(raw=True)
    Cps, conv = lat.get_deposit()
    lat.step(60)
    Cg, convg = lat.get_deposit()
    f, h = split_pops(p, lat.populations())
    print(storage, conv, convg, flush=True)
    assert conv > 0 and convg > conv
    assert np.isfinite(f).all() and np.isfinite(h).all() and np.isfinite(Cg).all()
    lat2 = mclbm.Lattice(p)
    lat2.set_geometry(m100)
    lat2.init_fields(rho, None, C)
    lat2.set_populations(pops, raw=True)
    lat2.set_deposit(Cps, conv)
    lat2.step(60)
    assert np.array_equal(lat.populations(raw=True), lat2.populations(raw=True))
    assert np.array_equal(lat.get_geometry()[0], lat2.get_geometry()[0])
    assert np.array_equal(Cg, lat2.get_deposit()[0])
    lat.close()
    lat2.close()
