"""GPU: the product species (CO2 made at the reacting walls, eq:react /
eq:reactCO2) against the FP64 oracle, through the C ABI.

Every population of both solute species within 1e-12 of the field's scale
(element by element) after tens of steps, in 3-D porous media with inlet/outlet and periodic solute, both forcing
schemes; the moments return both concentrations; a batch carries the product
per sample exactly as single runs do.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs

from helpers import gpu_lattice, maxrel, oracle_state, small_porous, split_pops

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("forcing", ["guo", "sc"])
@pytest.mark.parametrize("solute", ["inlet_outlet_x", "periodic"])
def test_product_populations_match_oracle(forcing, solute):
    p, mask, rho, u, C = small_porous(forcing=forcing, solute=solute, storage="f64",
                                      tau=(0.9, 1.3) if forcing == "sc" else (1.0, 1.0),
                                      k_wall=0.05, C_in=1.0, product=1, D2=0.17, C_in2=0.2)
    m, f, h = oracle_state(p, mask, rho, u, C)
    oracle.step(p, m, f, h, 40)
    lat = gpu_lattice(p, mask, rho, u, C)
    lat.step(40)
    fg, hg = split_pops(p, lat.populations())
    QS = 7
    print(forcing, solute, maxrel(fg, f), maxrel(hg[:QS], h[:QS]), maxrel(hg[QS:], h[QS:]), flush=True)
    assert hg.shape == h.shape == (2 * QS, f.shape[1])
    assert np.abs(h[QS:]).max() > 0          # the product exists
    assert maxrel(fg, f) < 1e-12
    assert maxrel(hg[:QS], h[:QS]) < 1e-12
    assert maxrel(hg[QS:], h[QS:]) < 1e-12
    _, _, Cg = lat.moments()
    _, _, Co = oracle.moments(p, m, f, h)
    assert Cg.shape == Co.shape == (2, f.shape[1])
    assert np.all(Cg[:, m.reshape(-1) != 0] == 0.0)      # solid nodes read 0 in both planes
    assert maxrel(Cg, Co) < 1e-12
    lat.close()


def test_product_in_a_2d_channel_and_fp32():
    """D2Q9 + two D2Q5 species, walls with reaction, inlet/outlet; FP64 over 300 steps,
    then FP32 one step from the same state within 2e-6 of the population scale."""
    nx, ny = 33, 17
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=ny, nz=1, ncomp=1, G=((0, 0), (0, 0)),
                           accel=(2e-5, 0, 0), solute="inlet_outlet_x", D=0.2, J0=0.4, k_wall=0.02, C_in=0.9,
                           product=1, D2=0.35, C_in2=0.0, storage="f64", tau=(0.8, 0.8))
    mask = np.zeros((1, ny, nx), np.uint8)
    mask[0, 0, :] = 1
    mask[0, ny - 1, :] = 1
    mask[0, 6:10, 12:15] = 1
    rho = np.where(mask == 0, 1.0, 0.0)[None]
    m, f, h = oracle_state(p, mask, rho)
    oracle.step(p, m, f, h, 300)
    lat = gpu_lattice(p, mask, rho)
    lat.step(300)
    fg, hg = split_pops(p, lat.populations())
    assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12
    lat.close()
    # FP32: load the FP64 state, one step, compare with the oracle's step from it
    p32 = dict(p, storage="f32")
    lat = gpu_lattice(p32, mask, rho)
    lat.set_populations(np.concatenate([f, h]).ravel())
    f32, h32 = split_pops(p32, lat.populations())
    f64, h64 = f32.copy(), h32.copy()
    oracle.step(p, m, f64, h64, 1)
    lat.step(1)
    fg, hg = split_pops(p32, lat.populations())
    scale = max(np.abs(f64).max(), np.abs(h64).max())
    assert np.abs(fg - f64).max() < 2e-6 * scale and np.abs(hg - h64).max() < 2e-6 * scale
    lat.close()


def test_product_batch_equals_single_runs():
    from paper_2502_12955_amd import mclbm

    cases = []
    for s, shape in enumerate([(10, 12, 14), (12, 10, 18)]):
        p, mask, rho, u, C = small_porous(shape=shape, seed_sample=20 + s, storage="f64", k_wall=0.05, C_in=1.0,
                                          product=1, D2=0.12, C_in2=0.1)
        cases.append((p, mask, rho, C))
    singles = []
    for p, mask, rho, C in cases:
        lat = gpu_lattice(p, mask, rho, None, C)
        lat.step(30)
        singles.append(lat.populations())
        lat.close()
    b = mclbm.Batch([c[0] for c in cases])
    b.set_geometry([c[1] for c in cases])
    b.init_fields([c[2] for c in cases], None, [c[3] for c in cases])
    b.step(30)
    pops = b.populations()
    off = 0
    for (p, _, _, _), ref in zip(cases, singles):
        got = pops[off: off + ref.size]
        off += ref.size
        assert np.array_equal(got, ref)
    b.close()


@pytest.mark.parametrize("product", [0, 1])
def test_rate_field_from_a_temperature_field_matches_oracle(product):
    """Arrhenius k(x) = A exp(-E / (R_u T(x))) of a prescribed temperature field: the
    reaction (and the product it makes) uses the rate of each wall node."""
    from paper_2502_12955_amd import mclbm

    p, mask, rho, u, C = small_porous(storage="f64", k_wall=0.0, C_in=1.0, product=product, D2=0.17,
                                      rate_field=1)
    shape = mask.shape
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    T = 700.0 + 15.0 * xx + 5.0 * np.sin(yy + zz)
    k_node = inputs.arrhenius_rate_field(T, 1.0, 2500.0).reshape(-1)
    assert 0.01 < k_node.min() and k_node.max() < 0.1
    po = dict(p, k_node=k_node)
    m, f, h = oracle_state(po, mask, rho, u, C)
    oracle.step(po, m, f, h, 40)
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    lat.set_wall_rate(k_node)
    lat.init_fields(rho, u, C)
    lat.step(40)
    fg, hg = split_pops(p, lat.populations())
    print(product, maxrel(fg, f), maxrel(hg, h), flush=True)
    assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12
    lat.close()
