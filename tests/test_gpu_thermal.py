"""GPU: conjugate heat transfer (Reactive LBM subsection) against the FP64 oracle.

The fluid and solid energy populations, the counter-slip interface solve with
the reaction heat and the C_b - T iteration run in the HIP library; the
oracle takes the same steps on the CPU.  Element by element, relative to each
field's scale: FP64 <= 1e-12 for the energy populations of fluid and solid,
the flow and solute populations and the temperature field, on a flat
reacting wall (D2Q9) and in a two-component 3-D sphere pack with the product
species and both forcing schemes.  FP32 against the FP64 oracle within 2e-5
(see the test).  Graph replay equals eager stepping bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs, mclbm

from helpers import maxrel, split_pops

pytestmark = pytest.mark.gpu


def _flat_wall(storage="f64"):
    p = inputs.base_params(lattice="D2Q9", nx=6, ny=24, nz=1, ncomp=1, G=((0, 0), (0, 0)), solute="periodic",
                           D=0.1, J0=0.4, k_wall=0.0, storage=storage)
    p.update(tau_ef=0.8, tau_es=1.2, rhocp_f=1.0, rhocp_s=2.0, h_r=0.8, arr_A=5.0, arr_E_over_R=2.0, T_tol=1e-14,
             T_maxit=100)
    mask = np.zeros((1, 24, 6), np.uint8)
    mask[0, :8, :] = 1
    N = mask.size
    rho = np.ones((1, N))
    C = np.ones(N)
    T = np.full(N, 1.0)
    return p, mask, rho, None, C, T


def _porous(storage="f64", forcing="guo"):
    shape = (12, 14, 16)
    p, mask, rho, u, C = inputs.porous_case(shape=shape, porosity=0.6, radius=3, blob_radius=2, sample=5,
                                           storage=storage)
    p.update(forcing=forcing, tau=(0.9, 1.3) if forcing == "sc" else (1.0, 1.0), solute="inlet_outlet_x",
             k_wall=0.0, C_in=1.0, product=1, D2=0.17, C_in2=0.1)
    p.update(tau_ef=0.85, tau_es=1.4, rhocp_f=1.0, rhocp_s=2.5, h_r=0.5, arr_A=3.0, arr_E_over_R=1.5,
             T_tol=1e-14, T_maxit=100)
    rng = inputs.SplitMix64(inputs.seed_for(9, 77))
    C = 0.5 * rng.uniform(int(np.prod(shape))).reshape(shape)
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    T = (1.0 + 0.05 * np.sin(0.4 * xx) + 0.03 * np.cos(0.3 * yy + 0.2 * zz)).reshape(-1)
    return p, mask, rho, u, C, T


def _run_both(p, mask, rho, u, C, T, steps):
    m, _ = oracle.pinch_fill(p, mask)
    f, h = oracle.init(p, m, rho, u, C)
    g, gs, Ti = oracle.thermal_init(p, m, T, u)
    ost = oracle.step_thermal(p, m, f, h, g, gs, Ti, steps)
    lat = mclbm.Lattice(p)
    lat.set_thermal(p)
    lat.set_geometry(mask)
    lat.init_fields(rho, u, C)
    lat.init_temperature(T, u)
    lat.step(steps)
    fg, hg = split_pops(p, lat.populations())
    gg, gsg = lat.thermal_populations()
    Tg = lat.temperature()
    gst = lat.thermal_stats()
    lat.close()
    To = oracle.temperature(p, m, g, gs)
    hs, it = oracle.thermal_nodes(p, m)
    fluid = m.reshape(-1) == 0
    holds = hs.astype(bool)
    return dict(f=(fg, f), h=(hg, h), g=(gg[:, fluid], g[:, fluid]), gs=(gsg[:, holds], gs[:, holds]),
                T=(Tg, To), stats=(gst, ost), it=it)


def test_flat_reacting_wall_fp64_matches_oracle():
    print("thermal: flat wall D2Q9 fp64, 60 steps", flush=True)
    r = _run_both(*_flat_wall(), steps=60)
    for key in ("f", "h", "g", "gs", "T"):
        a, b = r[key]
        err = maxrel(a, b)
        print(key, err, flush=True)
        assert err <= 1e-12, key
    gst, ost = r["stats"]
    assert gst[1] == 0 and ost[1] == 0 and gst[2] == ost[2] == 0
    assert abs(gst[0] - ost[0]) <= 0.01 * ost[0]


@pytest.mark.parametrize("forcing", ["guo", "sc"])
def test_porous_3d_fp64_matches_oracle(forcing):
    print(f"thermal: porous D3Q19 fp64 {forcing}, 30 steps", flush=True)
    r = _run_both(*_porous("f64", forcing), steps=30)
    for key in ("f", "h", "g", "gs", "T"):
        a, b = r[key]
        err = maxrel(a, b)
        print(key, err, flush=True)
        assert err <= 1e-12, key
    gst, ost = r["stats"]
    assert gst[2] == ost[2]            # degenerate interface nodes: a property of the geometry
    assert gst[1] == 0 and ost[1] == 0
    assert r["it"].sum() > 100


def test_porous_3d_fp32_within_tolerance():
    """FP32 storage and arithmetic against the FP64 oracle after 30 steps.  Each
    step rounds the populations to FP32 (relative 6e-8) and the interface
    iteration stops at 4 x 1.2e-7; over 30 steps of diffusion these stay below
    a few 1e-6 of the field scale, so 2e-5 bounds every field with margin."""
    print("thermal: porous D3Q19 fp32, 30 steps", flush=True)
    p, mask, rho, u, C, T = _porous("f32")
    r = _run_both(p, mask, rho, u, C, T, steps=30)
    for key in ("g", "gs", "T", "h"):
        a, b = r[key]
        err = maxrel(a, b)
        print(key, err, flush=True)
        assert err <= 2e-5, key


def test_thermal_graph_replay_equals_eager():
    print("thermal: graph replay vs eager", flush=True)
    p, mask, rho, u, C, T = _porous("f64")
    p["monitor_every"] = 10
    out = []
    for graph in (False, True):
        lat = mclbm.Lattice(p)
        lat.set_thermal(p)
        lat.set_geometry(mask)
        lat.init_fields(rho, u, C)
        lat.init_temperature(T, u)
        lat.set_graph(graph)
        lat.step(40)
        out.append((lat.populations(raw=True), lat.thermal_populations(), lat.temperature()))
        lat.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1][0], out[1][1][0]) and np.array_equal(out[0][1][1], out[1][1][1])
    assert np.array_equal(out[0][2], out[1][2])


def test_contact_temperature_on_the_gpu():
    """The GPU path reproduces the effusivity-weighted contact temperature of two
    half-spaces (t^-1/2 extrapolation from 400 and 1600 steps), as the oracle does."""
    print("thermal: contact temperature D2Q9 fp64", flush=True)
    p = inputs.base_params(lattice="D2Q9", nx=4, ny=600, nz=1, ncomp=1, G=((0, 0), (0, 0)), solute="off",
                           storage="f64")
    p.update(tau_ef=0.8, tau_es=1.3, rhocp_f=1.0, rhocp_s=2.5, h_r=0.0, T_tol=1e-14, T_maxit=100)
    mask = np.zeros((1, 600, 4), np.uint8)
    mask[0, :300, :] = 1
    N = mask.size
    lat = mclbm.Lattice(p)
    lat.set_thermal(p)
    lat.set_geometry(mask)
    lat.init_fields(np.ones((1, N)))
    lat.init_temperature(np.where(mask.reshape(-1) == 1, 1.0, 2.0))
    lat.step(400)
    T400 = lat.temperature().reshape(600, 4)[300, 0]
    lat.step(1200)
    T1600 = lat.temperature().reshape(600, 4)[300, 0]
    lat.close()
    ef, es = 1.0 * np.sqrt(0.3 / 3), 2.5 * np.sqrt(0.8 / 3)
    want = (ef * 2.0 + es * 1.0) / (ef + es)
    assert abs(2 * T1600 - T400 - want) < 1.5e-3


def test_thermal_argument_and_state_errors():
    p, mask, rho, u, C, T = _flat_wall()
    lat = mclbm.Lattice(p)
    with pytest.raises(mclbm.MclbmError):
        lat.set_thermal(dict(p, tau_ef=0.5))
    lat.set_thermal(p)
    lat.set_geometry(mask)
    lat.init_fields(rho, u, C)
    with pytest.raises(mclbm.MclbmError) as e:
        lat.step(1)                     # no temperature yet
    assert e.value.code == mclbm.ESTATE
    with pytest.raises(mclbm.MclbmError):
        lat.init_temperature(np.zeros(mask.size))   # T must be > 0
    lat.close()
    q = dict(p, storage="f16s")
    lat = mclbm.Lattice(q)
    with pytest.raises(mclbm.MclbmError):
        lat.set_thermal(q)
    lat.close()
